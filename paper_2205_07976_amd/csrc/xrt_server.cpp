// xrt_server.cpp -- continuous batching of served shots (host side).
//
// The paper runs many simulations per GPU and hides latency by letting several
// producers share one GPU (section IV, ranks per GPU).  Here one server owns a
// device arena (its HBM budget), admits submitted shots in arrival order as
// arena memory and resident slots allow, and feeds their tiles to a
// persistent kernel through a ring of chunks in pinned host memory:
//
//   submit    validate and copy the shot; queued (never blocks)
//   progress  (1) collect finished chunks from their done flags;
//             (2) admit queued shots: first-fit allocation of the image in
//                 the device arena and of descriptor + tables in a pinned
//                 host arena, written in place;
//             (3) publish chunks of the admitted shots, least work first, up to a
//                 bounded depth, then move the tail (release);
//             (4) launch the persistent kernel if none is running and
//                 published chunks wait.
//   image / release   read a finished image in place, then free its memory.
//
// Work of shots admitted while others run joins the same persistent kernel
// (continuous batching); every pixel is computed by the same arithmetic as
// xrt_simulate, so a shot's image does not depend on the mix it ran in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/xrt.h"
#include "xrt_internal.h"
#include "xrt_host.h"

using xrt::host::fail;
using xrt::host::hip_fail;

namespace {

constexpr uint64_t ALIGN = 256;
constexpr uint32_t RING = 1u << 16;
constexpr int TILE_PIXELS = 256;           // 16 x 16 pixels per tile
constexpr uint64_t CHUNK_TERMS = 1u << 20;  // pixel-terms a chunk aims at

uint64_t align_up(uint64_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// First-fit allocator over [0, size) with coalescing.
class Arena {
  public:
    explicit Arena(uint64_t size) { free_[0] = size; }
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

  private:
    std::map<uint64_t, uint64_t> free_;
};

struct Shot {
    uint64_t ticket = 0;
    int state = XRT_SHOT_QUEUED;
    xrt_detector det{};
    xrt_beam beam{};
    xrt_crystal xtal{};
    std::vector<double> dir, lam, weight, umats;
    uint64_t desc_bytes = 0, image_bytes = 0, part_bytes = 0, footprint = 0;
    uint64_t desc_off = 0, image_off = 0;  // in the host and device arenas
    int32_t n_tiles = 0, split = 1;
    uint64_t terms_per_pixel = 0;
    // the current phase: CHUNK_COMPUTE over units tile * split + part, then,
    // for split sums, CHUNK_REDUCE over tiles once every part is done
    int32_t phase = xrt::CHUNK_COMPUTE;
    int32_t n_units = 0, chunk_units = 1, next_unit = 0;
    int64_t chunks_total = 0, chunks_done = 0;
    double work_published = 0;  // pixel-terms of the chunks published so far
    double t_submit = 0, t_admit = -1, t_done = -1;
};

struct InFlight {
    uint64_t seq;
    uint64_t ticket;
};

}  // namespace

struct xrt_server {
    std::mutex mu;
    int device = 0;
    xrt_server_desc desc{};
    const xrt_fhkl *fhkl = nullptr;
    Arena *arena = nullptr;       // device arena: images (the HBM budget)
    Arena *harena = nullptr;      // host arena: descriptors and tables
    char *dev_arena = nullptr;
    char *host_arena = nullptr;
    uint64_t host_bytes = 0;
    // device control block: [0] chunks claimed, [1] time of the latest
    // finished chunk, then two 32-bit words: busy workgroups, exit flag
    unsigned long long *dev_ctl = nullptr;
    xrt::ServeCtrl *ctrl = nullptr;
    xrt::ServeChunk *ring = nullptr;
    uint32_t *done = nullptr;
    hipStream_t work = nullptr, copy = nullptr;
    hipEvent_t kernel_done = nullptr;
    bool launched = false;
    int n_wg = 0;
    uint64_t next_ticket = 1, tail = 0, resident = 0;
    std::deque<uint64_t> queue;                    // submitted, not admitted (FIFO)
    std::vector<uint64_t> admitted;                // admitted with tiles left to publish
    std::vector<InFlight> inflight;                // published chunks not yet done
    double vtime = 0;                              // published work of the shot served last
    std::unordered_map<uint64_t, Shot> shots;
    std::chrono::steady_clock::time_point t0;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

xrt_status check_desc(const xrt_server_desc *d)
{
    if (!d) return fail(XRT_EINVAL, "server descriptor is NULL");
    if (d->struct_size != sizeof(xrt_server_desc))
        return fail(XRT_EVERSION, "xrt_server_desc.struct_size %u, library expects %zu", d->struct_size,
                    sizeof(xrt_server_desc));
    if (d->hbm_budget < (1u << 20) || d->hbm_budget > ((uint64_t)1 << 40))
        return fail(XRT_ERANGE, "hbm_budget must be in [1 MiB, 1 TiB]");
    if (d->max_resident < 1 || d->max_resident > 65536) return fail(XRT_ERANGE, "max_resident must be in [1, 65536]");
    if (d->precision != XRT_FP64 && d->precision != XRT_MIXED) return fail(XRT_EINVAL, "unknown precision");
    if (d->shape != XRT_SHAPE_SINCG && d->shape != XRT_SHAPE_GAUSS) return fail(XRT_EINVAL, "unknown shape");
    if (d->out_dtype != XRT_F32 && d->out_dtype != XRT_F64) return fail(XRT_EINVAL, "unknown out_dtype");
    if (d->workgroups < 0 || d->workgroups > 65536) return fail(XRT_ERANGE, "workgroups must be in [0, 65536]");
    if (!(d->idle_exit_us >= 1.0 && d->idle_exit_us <= 1e6)) return fail(XRT_ERANGE, "idle_exit_us must be in [1, 1e6]");
    return XRT_OK;
}

void free_server(xrt_server *s)
{
    if (s->kernel_done) (void)hipEventDestroy(s->kernel_done);
    if (s->work) (void)hipStreamDestroy(s->work);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    if (s->dev_arena) (void)hipFree(s->dev_arena);
    if (s->dev_ctl) (void)hipFree(s->dev_ctl);
    if (s->ctrl) (void)hipHostFree(s->ctrl);
    if (s->ring) (void)hipHostFree(s->ring);
    if (s->done) (void)hipHostFree(s->done);
    if (s->host_arena) (void)hipHostFree(s->host_arena);
    delete s->arena;
    delete s->harena;
    delete s;
}

// Whether the persistent kernel still runs; a device error ends it too and
// is returned in *err.
bool kernel_running(xrt_server *s, hipError_t *err)
{
    *err = hipSuccess;
    if (!s->launched) return false;
    const hipError_t e = hipEventQuery(s->kernel_done);
    if (e == hipErrorNotReady) return true;
    s->launched = false;
    if (e != hipSuccess) *err = e;
    return false;
}

// Chunking of a shot's current phase.  Compute chunks hold about
// CHUNK_TERMS pixel-terms (a few ms of one workgroup, so a shot admitted later
// waits at most that long for a workgroup, and the last chunks of a shot end
// close together) and no more units than spread the phase over every
// workgroup; reduce chunks (K loads per pixel) are spread the same way.
void start_phase(xrt_server *s, Shot &sh, int32_t phase)
{
    sh.phase = phase;
    sh.n_units = phase == xrt::CHUNK_COMPUTE ? sh.n_tiles * sh.split : sh.n_tiles;
    const uint64_t by_spread = ((uint64_t)sh.n_units + s->n_wg - 1) / s->n_wg;
    uint64_t by_cost = (uint64_t)xrt::SERVE_MAX_CHUNK;
    if (phase == xrt::CHUNK_COMPUTE) {
        const uint64_t per_unit = std::max<uint64_t>(1, TILE_PIXELS * sh.terms_per_pixel / (uint64_t)sh.split);
        by_cost = std::max<uint64_t>(1, CHUNK_TERMS / per_unit);
    }
    sh.chunk_units = (int32_t)std::max<uint64_t>(
        1, std::min<uint64_t>({by_cost, by_spread, (uint64_t)xrt::SERVE_MAX_CHUNK}));
    sh.next_unit = 0;
    sh.chunks_total = (sh.n_units + sh.chunk_units - 1) / sh.chunk_units;
    sh.chunks_done = 0;
}

// (1) done flags -> finished chunks -> finished phases and shots.
void collect(xrt_server *s, int32_t *n_done)
{
    size_t w = 0;
    for (size_t i = 0; i < s->inflight.size(); ++i) {
        const InFlight f = s->inflight[i];
        const uint32_t flag = __atomic_load_n(&s->done[f.seq % RING], __ATOMIC_ACQUIRE);
        if (flag == (uint32_t)(f.seq + 1)) {
            Shot &sh = s->shots[f.ticket];
            if (++sh.chunks_done == sh.chunks_total) {
                if (sh.phase == xrt::CHUNK_COMPUTE && sh.split > 1) {
                    start_phase(s, sh, xrt::CHUNK_REDUCE);  // every part sum is in the arena
                    s->admitted.push_back(sh.ticket);
                } else {
                    sh.state = XRT_SHOT_DONE;
                    sh.t_done = s->now();
                    if (n_done) ++*n_done;
                }
            }
        } else {
            s->inflight[w++] = f;
        }
    }
    s->inflight.resize(w);
}

// (2) admission: device memory for the image, host memory for the
// descriptor and a resident slot, in arrival order.  The descriptor and tables
// are written straight into the pinned host arena: no device copy is needed,
// so admission never waits for the running persistent kernel.
xrt_status admit(xrt_server *s)
{
    while (!s->queue.empty() && s->resident < (uint64_t)s->desc.max_resident) {
        Shot &sh = s->shots[s->queue.front()];
        uint64_t doff = 0, hoff = 0;
        if (!s->arena->alloc(sh.footprint, &doff)) break;
        if (!s->harena->alloc(sh.desc_bytes, &hoff)) {
            s->arena->release(doff, sh.footprint);
            break;
        }
        sh.beam.dir = sh.dir.data();
        sh.beam.lambda = sh.lam.data();
        sh.beam.weight = sh.weight.data();
        sh.xtal.umats = sh.umats.data();
        std::vector<double> host;
        xrt::ShotDesc d;
        xrt_status st = xrt::host::served_descriptor(&sh.det, &sh.beam, &sh.xtal, s->fhkl, s->desc.out_dtype, &d, host);
        if (st) {
            s->arena->release(doff, sh.footprint);
            s->harena->release(hoff, sh.desc_bytes);
            return st;
        }
        d.mats_rel = align_up(sizeof(xrt::ShotDesc));
        d.src_rel = d.mats_rel + 9 * sizeof(double) * (size_t)d.p.n_rot;
        d.image_off = doff;
        d.image_bytes = sh.image_bytes;
        d.partial_off = doff + align_up(sh.image_bytes);
        d.partial_bytes = sh.part_bytes;
        if (d.p.split != sh.split) {
            s->arena->release(doff, sh.footprint);
            s->harena->release(hoff, sh.desc_bytes);
            return fail(XRT_EINVAL, "internal: split %d at admission, %d at submission", d.p.split, sh.split);
        }
        std::memcpy(s->host_arena + hoff, &d, sizeof d);
        std::memcpy(s->host_arena + hoff + d.mats_rel, host.data(), sizeof(double) * host.size());
        sh.desc_off = hoff;
        sh.image_off = doff;
        sh.state = XRT_SHOT_RUNNING;
        sh.t_admit = s->now();
        sh.n_tiles = d.p.n_tiles;
        sh.terms_per_pixel = (uint64_t)d.p.O * (uint64_t)d.p.O * (uint64_t)d.p.T * (uint64_t)d.p.n_src *
                             (uint64_t)d.p.n_rot;
        start_phase(s, sh, xrt::CHUNK_COMPUTE);
        sh.work_published = s->vtime;  // it competes from now on, not from the start
        s->resident++;
        s->admitted.push_back(sh.ticket);
        s->queue.pop_front();
    }
    return XRT_OK;
}

// (3) publication, while fewer than two chunks per workgroup are in flight:
// the next chunk always comes from the admitted shot with the least work
// published so far (pixel-terms; ties to the earlier ticket), so resident
// shots share the device evenly by work whatever their chunk sizes, and a
// small shot admitted later is not stuck behind a large one.  The shallow
// queue lets a newly admitted shot's chunks enter the ring as soon as earlier
// chunks finish.
void publish(xrt_server *s)
{
    const size_t depth = std::min<size_t>(RING - 1, 2 * (size_t)s->n_wg);
    bool any = false;
    while (s->inflight.size() < depth && !s->admitted.empty()) {
        size_t best = 0;
        for (size_t i = 1; i < s->admitted.size(); ++i) {
            const Shot &a = s->shots[s->admitted[i]], &b = s->shots[s->admitted[best]];
            if (a.work_published < b.work_published ||
                (a.work_published == b.work_published && a.ticket < b.ticket))
                best = i;
        }
        Shot &sh = s->shots[s->admitted[best]];
        s->vtime = sh.work_published;
        const uint64_t seq = s->tail;
        xrt::ServeChunk &c = s->ring[seq % RING];
        c.desc_off = sh.desc_off;
        c.tile0 = sh.next_unit;
        c.n_tiles = std::min(sh.chunk_units, sh.n_units - sh.next_unit);
        c.seq1 = (uint32_t)(seq + 1);
        c.shot = (uint32_t)sh.ticket ? (uint32_t)sh.ticket : 1u;
        c.kind = sh.phase;
        c.pad = 0;
        sh.next_unit += c.n_tiles;
        // a reduce chunk reads K values per pixel: count it as K terms
        sh.work_published += (double)c.n_tiles * TILE_PIXELS *
                             (sh.phase == xrt::CHUNK_COMPUTE ? (double)sh.terms_per_pixel / sh.split : sh.split);
        s->inflight.push_back({seq, sh.ticket});
        s->tail++;
        any = true;
        if (sh.next_unit >= sh.n_units) s->admitted.erase(s->admitted.begin() + best);
    }
    if (any) __atomic_store_n(&s->ctrl->tail, s->tail, __ATOMIC_RELEASE);
}

xrt_status launch(xrt_server *s)
{
    hipError_t err;
    const bool running = kernel_running(s, &err);
    if (err != hipSuccess) return hip_fail(err, "xrt_server_progress: persistent kernel");
    if (s->inflight.empty() || running) return XRT_OK;
    xrt::ServeArgs a{};
    a.ctrl = s->ctrl;
    a.ring = s->ring;
    a.done = s->done;
    a.cap = RING;
    a.next = s->dev_ctl;
    a.last_done = s->dev_ctl + 1;
    a.busy = reinterpret_cast<unsigned int *>(s->dev_ctl + 2);
    a.exiting = a.busy + 1;
    a.hdesc = s->host_arena;
    a.hdesc_bytes = s->host_bytes;
    a.arena = s->dev_arena;
    a.arena_bytes = s->desc.hbm_budget;
    xrt::host::fhkl_tables(s->fhkl, &a.F2_64, &a.F2_32, &a.bytes64, &a.bytes32);
    a.idle_ticks = (uint64_t)(s->desc.idle_exit_us * 100.0);  // s_memrealtime: 100 MHz
    // a new kernel starts with no busy workgroup, no exit flag, no finished chunk
    hipError_t e = hipMemsetAsync(s->dev_ctl + 1, 0, 2 * sizeof(unsigned long long), s->work);
    if (e == hipSuccess) e = xrt::launch_serve(a, s->desc.precision, s->desc.shape, s->n_wg, s->work);
    if (e == hipSuccess) e = hipEventRecord(s->kernel_done, s->work);
    if (e != hipSuccess) return hip_fail(e, "xrt_server_progress: launch");
    s->launched = true;
    return XRT_OK;
}

}  // namespace

extern "C" {

xrt_status xrt_server_create(const xrt_server_desc *desc, const xrt_fhkl *fhkl, xrt_server **out)
{
    xrt_status st;
    if (!out) return fail(XRT_EINVAL, "NULL output pointer");
    *out = nullptr;
    if ((st = check_desc(desc))) return st;
    if (!fhkl) return fail(XRT_EINVAL, "fhkl is NULL");
    xrt_server *s = new (std::nothrow) xrt_server();
    if (!s) return fail(XRT_ENOMEM, "host allocation failed");
    s->desc = *desc;
    s->fhkl = fhkl;
    s->t0 = std::chrono::steady_clock::now();
    hipError_t e = hipGetDevice(&s->device);
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device);
    // as many workgroups as the device holds at once, less eight: the free
    // slots let small kernels (result copies) run beside the persistent one
    const int per_cu = e == hipSuccess ? xrt::serve_blocks_per_cu(desc->precision, desc->shape) : 0;
    if (e == hipSuccess && per_cu < 1) e = hipErrorInvalidConfiguration;
    s->n_wg = desc->workgroups ? desc->workgroups : std::max(per_cu * std::max(cus, 1) - 8, 1);
    s->host_bytes = (uint64_t)std::min(desc->max_resident, 4096) * (32u << 10);
    if (e == hipSuccess) e = hipMalloc((void **)&s->dev_arena, desc->hbm_budget);
    if (e == hipSuccess) e = hipMalloc((void **)&s->dev_ctl, 4 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(s->dev_ctl, 0, 4 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->ctrl, sizeof(xrt::ServeCtrl), hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->ring, sizeof(xrt::ServeChunk) * RING, hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->done, sizeof(uint32_t) * RING, hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->host_arena, s->host_bytes, hipHostMallocCoherent);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->work, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->kernel_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_server(s);
        return hip_fail(e, "xrt_server_create");
    }
    std::memset(s->ctrl, 0, sizeof(xrt::ServeCtrl));
    std::memset(s->ring, 0, sizeof(xrt::ServeChunk) * RING);
    std::memset(s->done, 0, sizeof(uint32_t) * RING);
    s->arena = new (std::nothrow) Arena(desc->hbm_budget);
    s->harena = new (std::nothrow) Arena(s->host_bytes);
    if (!s->arena || !s->harena) {
        free_server(s);
        return fail(XRT_ENOMEM, "host allocation failed");
    }
    *out = s;
    return XRT_OK;
}

xrt_status xrt_server_destroy(xrt_server *s)
{
    if (!s) return XRT_OK;
    hipError_t e = hipSuccess;
    {
        std::lock_guard<std::mutex> g(s->mu);
        __atomic_store_n(&s->ctrl->stop, 1u, __ATOMIC_RELEASE);
        if (s->launched) e = hipEventSynchronize(s->kernel_done);
        if (e == hipSuccess) e = hipStreamSynchronize(s->copy);
    }
    free_server(s);
    if (e != hipSuccess) return hip_fail(e, "xrt_server_destroy");
    return XRT_OK;
}

xrt_status xrt_server_submit(xrt_server *s, const xrt_detector *det, const xrt_beam *beam, const xrt_crystal *xtal,
                             uint64_t *ticket)
{
    if (!s || !ticket) return fail(XRT_EINVAL, "NULL argument");
    xrt_status st;
    if ((st = xrt::host::check_shot(det, beam, xtal))) return st;
    if (xtal->shape != s->desc.shape) return fail(XRT_EINVAL, "shot shape differs from the server's");
    if ((int64_t)xtal->n_phi * xtal->n_mos > xrt::SERVE_MAX_ROT)
        return fail(XRT_ERANGE, "served shots take at most %d spindle steps x domains", xrt::SERVE_MAX_ROT);
    if (beam->n_src > xrt::SERVE_MAX_SRC)
        return fail(XRT_ERANGE, "served shots take at most %d sources", xrt::SERVE_MAX_SRC);
    Shot sh;
    sh.det = *det;
    sh.beam = *beam;
    sh.xtal = *xtal;
    sh.dir.assign(beam->dir, beam->dir + 3 * beam->n_src);
    sh.lam.assign(beam->lambda, beam->lambda + beam->n_src);
    sh.weight.assign(beam->weight, beam->weight + beam->n_src);
    sh.umats.assign(xtal->umats, xtal->umats + 9 * (size_t)xtal->n_mos);
    const uint64_t n_pix = (uint64_t)(det->roi_f1 - det->roi_f0) * (uint64_t)(det->roi_s1 - det->roi_s0);
    const uint64_t tables = sizeof(double) * (9 * (uint64_t)xtal->n_phi * xtal->n_mos + xrt::SRC_STRIDE * (uint64_t)beam->n_src);
    sh.desc_bytes = align_up(align_up(sizeof(xrt::ShotDesc)) + tables);
    sh.image_bytes = n_pix * (s->desc.out_dtype == XRT_F64 ? 8 : 4);
    // split sums keep their part sums in the arena after the image
    sh.split = xrt::host::split_of(det, beam, xtal);
    const uint64_t n_tiles = (uint64_t)((det->roi_f1 - det->roi_f0 + 15) / 16) *
                             (uint64_t)((det->roi_s1 - det->roi_s0 + 15) / 16);
    sh.part_bytes = sh.split > 1 ? sizeof(double) * n_tiles * (uint64_t)sh.split * TILE_PIXELS : 0;
    sh.footprint = align_up(sh.image_bytes) + align_up(sh.part_bytes);
    if (sh.footprint > s->desc.hbm_budget)
        return fail(XRT_ERANGE, "shot needs %llu bytes, more than the server's budget %llu",
                    (unsigned long long)sh.footprint, (unsigned long long)s->desc.hbm_budget);
    std::lock_guard<std::mutex> g(s->mu);
    sh.ticket = s->next_ticket++;
    sh.t_submit = s->now();
    *ticket = sh.ticket;
    s->queue.push_back(sh.ticket);
    s->shots.emplace(sh.ticket, std::move(sh));
    return XRT_OK;
}

xrt_status xrt_server_progress(xrt_server *s, int32_t *n_done)
{
    if (!s) return fail(XRT_EINVAL, "server is NULL");
    if (n_done) *n_done = 0;
    std::lock_guard<std::mutex> g(s->mu);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != s->device) return fail(XRT_EINVAL, "server lives on device %d, current device is %d", s->device, dev);
    collect(s, n_done);
    xrt_status st = admit(s);
    if (st) return st;
    publish(s);
    // a kernel that ended (idle exit) is relaunched when published work waits
    return launch(s);
}

xrt_status xrt_server_info(xrt_server *s, uint64_t ticket, xrt_shot_info *info)
{
    if (!s || !info) return fail(XRT_EINVAL, "NULL argument");
    if (info->struct_size != sizeof(xrt_shot_info))
        return fail(XRT_EVERSION, "xrt_shot_info.struct_size %u, library expects %zu", info->struct_size,
                    sizeof(xrt_shot_info));
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->shots.find(ticket);
    if (it == s->shots.end()) return fail(XRT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    const Shot &sh = it->second;
    info->state = sh.state;
    info->image_bytes = sh.image_bytes;
    info->roi_nf = sh.det.roi_f1 - sh.det.roi_f0;
    info->roi_ns = sh.det.roi_s1 - sh.det.roi_s0;
    info->t_submit = sh.t_submit;
    info->t_admit = sh.t_admit;
    info->t_done = sh.t_done;
    return XRT_OK;
}

xrt_status xrt_server_image(xrt_server *s, uint64_t ticket, const void **dev_image)
{
    if (!s || !dev_image) return fail(XRT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->shots.find(ticket);
    if (it == s->shots.end()) return fail(XRT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second.state != XRT_SHOT_DONE) return fail(XRT_EBUSY, "shot %llu is not done", (unsigned long long)ticket);
    *dev_image = s->dev_arena + it->second.image_off;
    return XRT_OK;
}

xrt_status xrt_server_release(xrt_server *s, uint64_t ticket)
{
    if (!s) return fail(XRT_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->shots.find(ticket);
    if (it == s->shots.end()) return fail(XRT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (it->second.state != XRT_SHOT_DONE) return fail(XRT_EBUSY, "shot %llu is not done", (unsigned long long)ticket);
    s->arena->release(it->second.image_off, it->second.footprint);
    s->harena->release(it->second.desc_off, it->second.desc_bytes);
    s->resident--;
    s->shots.erase(it);
    return XRT_OK;
}

}  // extern "C"
