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
// With write-out (a host budget), a shot that finishes on the device is
// copied into pinned host memory on a copy stream while the persistent kernel
// goes on with other shots; once the copy is complete the shot's device memory
// and resident slot are freed and the shot is reported done, so admission
// never waits for a client that is still writing earlier images out.
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
#include "xrt_host.h"
#include "xrt_internal.h"
#include "xrt_sched.h"

using xrt::host::fail;
using xrt::host::hip_fail;

namespace {

using xrt::sched::align_up;
constexpr uint32_t RING = xrt::SERVE_RING;
static_assert(xrt::sched::PHASE_COMPUTE == xrt::CHUNK_COMPUTE && xrt::sched::PHASE_REDUCE == xrt::CHUNK_REDUCE &&
                  xrt::sched::PHASE_BACKGROUND == xrt::CHUNK_BACKGROUND,
              "chunk kinds");
static_assert(xrt::sched::MAX_CHUNK == xrt::SERVE_MAX_CHUNK, "units per chunk");
static_assert(xrt::sched::TILE_PIXELS == 256, "tile of the kernels");
static_assert(xrt::sched::QUEUED == XRT_SHOT_QUEUED && xrt::sched::RUNNING == XRT_SHOT_RUNNING &&
                  xrt::sched::DONE == XRT_SHOT_DONE,
              "shot states");

// What the server keeps of a shot beside the scheduler's record: the shot
// itself (read again at admission), its image size and its times.
struct Shot {
    xrt_detector det{};
    xrt_beam beam{};
    xrt_crystal xtal{};
    std::vector<double> dir, lam, weight, umats;
    uint64_t image_bytes = 0, part_bytes = 0, state_bytes = 0;
    double t_submit = 0, t_admit = -1, t_done = -1;
    // write-out: the image's place in the host arena and the copy's event;
    // written once the copy has completed (the device memory is gone then)
    uint64_t out_off = 0;
    hipEvent_t copied = nullptr;
    bool written = false;
};

}  // namespace

struct xrt_server {
    std::mutex mu;
    int device = 0;
    xrt_server_desc desc{};
    const xrt_fhkl *fhkl = nullptr;
    xrt::sched::Scheduler *sched = nullptr;  // arenas, admission, chunks, publication order
    char *dev_arena = nullptr;               // images and part sums (the HBM budget)
    char *host_arena = nullptr;              // descriptors and tables (pinned)
    uint64_t host_bytes = 0;
    // device control block: [0] chunks claimed, [1] time of the latest
    // finished chunk, then two 32-bit words: busy workgroups, exit flag
    unsigned long long *dev_ctl = nullptr;
    xrt::ServeCtrl *ctrl = nullptr;
    xrt::ServeChunk *ring = nullptr;
    uint32_t *done = nullptr;
    hipStream_t work = nullptr;              // the persistent kernel's stream
    hipEvent_t kernel_done = nullptr;
    // write-out (desc.host_budget > 0): pinned host arena of finished images,
    // the copy stream, shots finished on the device that wait for host space
    // (in finishing order), copies in flight, and spare events
    char *out = nullptr;
    xrt::sched::Arena *out_arena = nullptr;
    hipStream_t copy = nullptr;
    // background (desc.background): the curve as BgKnot records of the
    // server's precision in device memory, and the molecule count
    void *bg_knots = nullptr;
    double bg_molecules = 0.0;
    std::deque<uint64_t> to_copy;
    std::vector<uint64_t> copying;
    std::vector<hipEvent_t> spare_events;
    bool launched = false;
    int n_wg = 0;
    uint64_t next_ticket = 1;
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
    if (d->host_budget != 0 && (d->host_budget < (1u << 20) || d->host_budget > ((uint64_t)1 << 40)))
        return fail(XRT_ERANGE, "host_budget must be 0 or in [1 MiB, 1 TiB]");
    if (d->policy != XRT_SERVE_FAIR_SHARE && d->policy != XRT_SERVE_SHORTEST_REMAINING)
        return fail(XRT_EINVAL, "unknown policy %d", d->policy);
    if (d->segment_terms != 0 && (d->segment_terms < (1 << 10) || d->segment_terms > ((int64_t)1 << 40)))
        return fail(XRT_ERANGE, "segment_terms must be 0 or in [2^10, 2^40]");
    if (d->background) return xrt::host::check_background_desc(d->background);
    return XRT_OK;
}

void free_server(xrt_server *s)
{
    if (s->copy) (void)hipStreamSynchronize(s->copy);
    for (auto &kv : s->shots)
        if (kv.second.copied) (void)hipEventDestroy(kv.second.copied);
    for (hipEvent_t e : s->spare_events) (void)hipEventDestroy(e);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    if (s->out) (void)hipHostFree(s->out);
    if (s->bg_knots) (void)hipFree(s->bg_knots);
    delete s->out_arena;
    if (s->kernel_done) (void)hipEventDestroy(s->kernel_done);
    if (s->work) (void)hipStreamDestroy(s->work);
    if (s->dev_arena) (void)hipFree(s->dev_arena);
    if (s->dev_ctl) (void)hipFree(s->dev_ctl);
    if (s->ctrl) (void)hipHostFree(s->ctrl);
    if (s->ring) (void)hipHostFree(s->ring);
    if (s->done) (void)hipHostFree(s->done);
    if (s->host_arena) (void)hipHostFree(s->host_arena);
    delete s->sched;
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

// Write-out: copies of finished shots into the host arena, in finishing
// order, as far as host space allows (the first that does not fit waits for
// releases, and the ones behind it wait too).
xrt_status start_copies(xrt_server *s)
{
    while (!s->to_copy.empty()) {
        const uint64_t t = s->to_copy.front();
        Shot &sh = s->shots[t];
        const xrt::sched::Work *w = s->sched->find(t);
        uint64_t off = 0;
        if (!s->out_arena->alloc(align_up(sh.image_bytes), &off)) break;
        hipEvent_t ev = nullptr;
        hipError_t e = hipSuccess;
        if (!s->spare_events.empty()) {
            ev = s->spare_events.back();
            s->spare_events.pop_back();
        } else {
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        }
        // the kernel wrote the image and made it visible at system scope
        // before raising the done flags that finished this shot
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->out + off, s->dev_arena + w->dev_off, sh.image_bytes, hipMemcpyDeviceToHost, s->copy);
        if (e == hipSuccess) e = hipEventRecord(ev, s->copy);
        if (e != hipSuccess) {
            s->out_arena->release(off, align_up(sh.image_bytes));
            if (ev) s->spare_events.push_back(ev);
            return hip_fail(e, "xrt_server_progress: image copy");
        }
        sh.out_off = off;
        sh.copied = ev;
        s->copying.push_back(t);
        s->to_copy.pop_front();
    }
    return XRT_OK;
}

// Write-out: completed copies free the shot's device memory and slot and make
// it done.  Returns the number of shots finished so.
xrt_status finish_copies(xrt_server *s, int32_t *n)
{
    size_t k = 0;
    for (size_t i = 0; i < s->copying.size(); ++i) {
        const uint64_t t = s->copying[i];
        Shot &sh = s->shots[t];
        const hipError_t e = hipEventQuery(sh.copied);
        if (e == hipErrorNotReady) {
            s->copying[k++] = t;
            continue;
        }
        if (e != hipSuccess) return hip_fail(e, "xrt_server_progress: image copy");
        s->spare_events.push_back(sh.copied);
        sh.copied = nullptr;
        sh.written = true;
        sh.t_done = s->now();
        s->sched->release(t);
        ++*n;
    }
    s->copying.resize(k);
    return XRT_OK;
}

// (1) done flags -> finished chunks -> finished phases and shots; with
// write-out, finished shots go to the copy queue and completed copies finish
// them.
xrt_status collect(xrt_server *s, int32_t *n_done)
{
    std::vector<uint64_t> finished;
    s->sched->collect([s](uint64_t seq) { return __atomic_load_n(&s->done[seq % RING], __ATOMIC_ACQUIRE) == (uint32_t)(seq + 1); },
                      &finished);
    int32_t n = 0;
    if (!s->out) {
        for (uint64_t t : finished) s->shots[t].t_done = s->now();
        n = (int32_t)finished.size();
    } else {
        for (uint64_t t : finished) s->to_copy.push_back(t);
        xrt_status st = finish_copies(s, &n);
        if (!st) st = start_copies(s);
        if (st) return st;
    }
    if (n_done) *n_done = n;
    return XRT_OK;
}

// (2) admission (in arrival order, by device-arena footprint and resident
// slots; the scheduler's rule): the descriptor and tables are written straight
// into the pinned host arena, so admission needs no device copy and never
// waits for the running persistent kernel.
xrt_status admit(xrt_server *s)
{
    return (xrt_status)s->sched->admit([s](xrt::sched::Work &w) -> int {
        Shot &sh = s->shots[w.ticket];
        sh.beam.dir = sh.dir.data();
        sh.beam.lambda = sh.lam.data();
        sh.beam.weight = sh.weight.data();
        sh.xtal.umats = sh.umats.data();
        std::vector<double> host;
        xrt::ShotDesc d;
        xrt_status st = xrt::host::served_descriptor(&sh.det, &sh.beam, &sh.xtal, s->fhkl, s->desc.out_dtype, &d, host);
        if (st) return st;
        if (d.p.split != w.split || d.p.n_tiles != w.n_tiles)
            return fail(XRT_EINVAL, "internal: shot plan differs between submission and admission");
        d.mats_rel = align_up(sizeof(xrt::ShotDesc));
        d.src_rel = d.mats_rel + 9 * sizeof(double) * (size_t)d.p.n_rot;
        d.image_off = w.dev_off;
        d.image_bytes = sh.image_bytes;
        d.partial_off = w.dev_off + align_up(sh.image_bytes);
        d.partial_bytes = sh.part_bytes;
        d.n_seg = w.n_seg;
        d.state_off = d.partial_off + align_up(sh.part_bytes);
        d.state_bytes = sh.state_bytes;
        d.bg_norm = s->bg_knots ? xrt::host::background_norm(&sh.det, &sh.beam, s->bg_molecules) : 0.0;
        std::memcpy(s->host_arena + w.host_off, &d, sizeof d);
        std::memcpy(s->host_arena + w.host_off + d.mats_rel, host.data(), sizeof(double) * host.size());
        sh.t_admit = s->now();
        return XRT_OK;
    });
}

// (3) publication (the scheduler's order and depth) into the ring, then the
// tail moves (release): the kernel may claim the new chunks from then on.
void publish(xrt_server *s)
{
    const size_t n = s->sched->publish([s](const xrt::sched::Chunk &k, const xrt::sched::Work &w) {
        xrt::ServeChunk &c = s->ring[k.seq % RING];
        c.desc_off = w.host_off;
        c.tile0 = k.unit0;
        c.n_tiles = k.n_units;
        c.seq1 = (uint32_t)(k.seq + 1);
        c.shot = (uint32_t)w.ticket ? (uint32_t)w.ticket : 1u;
        c.kind = k.kind;
        c.seg = k.seg;
    });
    if (n) __atomic_store_n(&s->ctrl->tail, s->sched->published(), __ATOMIC_RELEASE);
}

xrt_status launch(xrt_server *s)
{
    hipError_t err;
    const bool running = kernel_running(s, &err);
    if (err != hipSuccess) return hip_fail(err, "xrt_server_progress: persistent kernel");
    if (s->sched->in_flight() == 0 || running) return XRT_OK;
    xrt::ServeArgs a{};
    a.ctrl = s->ctrl;
    a.ring = s->ring;
    a.done = s->done;
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
    a.bg_knots = s->bg_knots;
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
    if (e == hipSuccess && desc->host_budget) {
        e = hipHostMalloc((void **)&s->out, desc->host_budget, hipHostMallocDefault);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
    }
    if (e == hipSuccess && desc->background) {
        // one record per interval (knot, next knot or NaN, F, slope), the
        // values the standalone background kernel stages from the same rows
        const int n = desc->background->n_knots;
        std::vector<double> k64(3 * (size_t)n), r64(4 * (size_t)n);
        std::vector<float> k32(3 * (size_t)n), r32(4 * (size_t)n);
        xrt::host::background_rows(desc->background, k64.data(), k32.data());
        for (int k = 0; k < n; ++k) {
            r64[4 * k] = k64[3 * k];
            r64[4 * k + 1] = k + 1 < n ? k64[3 * k + 3] : std::nan("");
            r64[4 * k + 2] = k64[3 * k + 1];
            r64[4 * k + 3] = k64[3 * k + 2];
            r32[4 * k] = k32[3 * k];
            r32[4 * k + 1] = k + 1 < n ? k32[3 * k + 3] : std::nanf("");
            r32[4 * k + 2] = k32[3 * k + 1];
            r32[4 * k + 3] = k32[3 * k + 2];
        }
        const bool f64 = desc->precision == XRT_FP64;
        const size_t bytes = f64 ? sizeof(double) * r64.size() : sizeof(float) * r32.size();
        e = hipMalloc(&s->bg_knots, bytes);
        if (e == hipSuccess)
            e = hipMemcpy(s->bg_knots, f64 ? (const void *)r64.data() : (const void *)r32.data(), bytes,
                          hipMemcpyHostToDevice);
        s->bg_molecules = desc->background->molecules;
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->kernel_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_server(s);
        return hip_fail(e, "xrt_server_create");
    }
    std::memset(s->ctrl, 0, sizeof(xrt::ServeCtrl));
    std::memset(s->ring, 0, sizeof(xrt::ServeChunk) * RING);
    std::memset(s->done, 0, sizeof(uint32_t) * RING);
    s->sched = new (std::nothrow) xrt::sched::Scheduler(
        desc->hbm_budget, s->host_bytes, desc->max_resident, s->n_wg, RING,
        desc->policy == XRT_SERVE_SHORTEST_REMAINING ? xrt::sched::POLICY_SHORTEST_REMAINING
                                                     : xrt::sched::POLICY_FAIR_SHARE);
    if (s->out) s->out_arena = new (std::nothrow) xrt::sched::Arena(desc->host_budget);
    if (!s->sched || (s->out && !s->out_arena)) {
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
    xrt::sched::Work w;
    const uint64_t n_pix = (uint64_t)(det->roi_f1 - det->roi_f0) * (uint64_t)(det->roi_s1 - det->roi_s0);
    const uint64_t tables = sizeof(double) * (9 * (uint64_t)xtal->n_phi * xtal->n_mos + xrt::SRC_STRIDE * (uint64_t)beam->n_src);
    w.desc_bytes = align_up(align_up(sizeof(xrt::ShotDesc)) + tables);
    sh.image_bytes = n_pix * (s->desc.out_dtype == XRT_F64 ? 8 : 4);
    // split sums keep their part sums in the arena after the image
    w.split = xrt::host::split_of(det, beam, xtal);
    w.n_tiles = (int32_t)(((det->roi_f1 - det->roi_f0 + 15) / 16) * ((det->roi_s1 - det->roi_s0 + 15) / 16));
    w.terms_per_pixel = (uint64_t)det->oversample * det->oversample * det->n_layers * (uint64_t)beam->n_src *
                        (uint64_t)xtal->n_phi * xtal->n_mos;
    if (s->bg_knots)  // the server's background, a phase after the sums
        w.bg_terms_per_pixel = (uint64_t)det->oversample * det->oversample * det->n_layers * (uint64_t)beam->n_src;
    sh.part_bytes = w.split > 1 ? sizeof(double) * (uint64_t)w.n_tiles * (uint64_t)w.split * xrt::sched::TILE_PIXELS : 0;
    // heavy units run as consecutive segments, their running sums kept in
    // the arena between two (8 bytes per unit and lane)
    const int64_t n_outer = (int64_t)det->oversample * det->oversample * det->n_layers * beam->n_src;
    w.n_seg = xrt::sched::segments_of(w.terms_per_pixel, w.split, n_outer,
                                      s->desc.segment_terms ? (uint64_t)s->desc.segment_terms
                                                            : xrt::sched::SEGMENT_TERMS);
    sh.state_bytes = w.n_seg > 1 ? 8 * (uint64_t)w.n_tiles * (uint64_t)w.split * xrt::sched::TILE_PIXELS : 0;
    w.footprint = align_up(sh.image_bytes) + align_up(sh.part_bytes) + align_up(sh.state_bytes);
    if (w.footprint > s->desc.hbm_budget)
        return fail(XRT_ERANGE, "shot needs %llu bytes, more than the server's budget %llu",
                    (unsigned long long)w.footprint, (unsigned long long)s->desc.hbm_budget);
    if (s->desc.host_budget && align_up(sh.image_bytes) > s->desc.host_budget)
        return fail(XRT_ERANGE, "image of %llu bytes exceeds the server's host budget %llu",
                    (unsigned long long)sh.image_bytes, (unsigned long long)s->desc.host_budget);
    std::lock_guard<std::mutex> g(s->mu);
    w.ticket = s->next_ticket++;
    sh.t_submit = s->now();
    *ticket = w.ticket;
    s->shots.emplace(w.ticket, std::move(sh));
    s->sched->submit(w);
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
    xrt_status st = collect(s, n_done);
    if (st) return st;
    st = admit(s);
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
    const xrt::sched::Work *w = s->sched->find(ticket);
    // with write-out a shot is done once its image is on the host (the
    // scheduler has forgotten it by then); until then it is running
    info->state = w ? (s->out && w->state == xrt::sched::DONE ? XRT_SHOT_RUNNING : w->state) : XRT_SHOT_DONE;
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
    if (s->out) return fail(XRT_EINVAL, "this server writes images out: use xrt_server_host_image");
    const xrt::sched::Work *w = s->sched->find(ticket);
    if (!w) return fail(XRT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (w->state != xrt::sched::DONE) return fail(XRT_EBUSY, "shot %llu is not done", (unsigned long long)ticket);
    *dev_image = s->dev_arena + w->dev_off;
    return XRT_OK;
}

xrt_status xrt_server_host_image(xrt_server *s, uint64_t ticket, const void **host_image)
{
    if (!s || !host_image) return fail(XRT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    if (!s->out) return fail(XRT_EINVAL, "this server has no host budget: use xrt_server_image");
    auto it = s->shots.find(ticket);
    if (it == s->shots.end()) return fail(XRT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second.written) return fail(XRT_EBUSY, "shot %llu is not done", (unsigned long long)ticket);
    *host_image = s->out + it->second.out_off;
    return XRT_OK;
}

xrt_status xrt_server_cancel(xrt_server *s, uint64_t ticket)
{
    if (!s) return fail(XRT_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    const xrt::sched::Work *w = s->sched->find(ticket);
    if (!w && s->shots.count(ticket))  // written out: done
        return fail(XRT_EBUSY, "shot %llu is already done", (unsigned long long)ticket);
    if (!w) return fail(XRT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (w->state != xrt::sched::QUEUED)
        return fail(XRT_EBUSY, "shot %llu is already admitted", (unsigned long long)ticket);
    s->sched->cancel(ticket);
    s->shots.erase(ticket);
    return XRT_OK;
}

xrt_status xrt_server_release(xrt_server *s, uint64_t ticket)
{
    if (!s) return fail(XRT_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    if (s->out) {
        auto it = s->shots.find(ticket);
        if (it == s->shots.end()) return fail(XRT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        if (!it->second.written) return fail(XRT_EBUSY, "shot %llu is not done", (unsigned long long)ticket);
        s->out_arena->release(it->second.out_off, align_up(it->second.image_bytes));
        s->shots.erase(it);
        return XRT_OK;
    }
    const xrt::sched::Work *w = s->sched->find(ticket);
    if (!w) return fail(XRT_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (w->state != xrt::sched::DONE) return fail(XRT_EBUSY, "shot %llu is not done", (unsigned long long)ticket);
    s->sched->release(ticket);
    s->shots.erase(ticket);
    return XRT_OK;
}

}  // extern "C"
