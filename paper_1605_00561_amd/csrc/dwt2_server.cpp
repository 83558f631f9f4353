// dwt2_server.cpp -- the serving loop of libdwt2 (declared in include/dwt2.h):
// requests from any host thread are grouped into batched transforms
// (continuous batching) on the caller's stream.
//
// Threads.  A scheduler forms each batch from the pending requests, in
// submission order, when fewer than max_inflight batches are on the stream:
// it stops at max_batch requests, at the first request whose buffers overlap
// one already taken (such a request must run after it), or at the first one
// whose workspace does not fit the free part of the arena.  It launches the
// forward and the inverse group of the batch (dwt2_forward_batch /
// dwt2_inverse_batch) and records an event.  The two groups touch disjoint
// memory, so when a batch has both, the inverse group runs on a second
// stream forked from the caller's stream and joined back into it: each
// group's latency-bound deep levels overlap the other group's work, and the
// order against earlier and later work on the caller's stream is unchanged.
// A completer waits for the oldest batch's event, stamps its requests and
// frees its arena block.
//
// Admission is by HBM footprint: a batch's workspace must fit a free block of
// the arena, and, when the caller sets a footprint cap, the requests in
// flight (launched, not yet retired) may together touch at most that many
// bytes of device memory, counting each request's input, output and LL
// buffers.
//
// The arena is a caller-owned device buffer; the server keeps only a host-side
// free list over it (first fit, coalescing), so nothing is allocated on the
// device.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/dwt2.h"
#include "dwt2_internal.h"
#include "server_plan.h"

#define DWT2_EXPORT extern "C" __attribute__((visibility("default")))

namespace {

using Clock = std::chrono::steady_clock;
constexpr size_t kAlign = 256;

double us_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::micro>(b - a).count();
}

size_t span_bytes(ptrdiff_t pitch, int w, int h)
{
    return sizeof(float) * ((size_t)(h - 1) * (size_t)pitch + (size_t)w);
}

using dwt2::serve::Arena;
using dwt2::serve::Group;

struct Pending {
    unsigned long long ticket;
    dwt2_request r;
    size_t ll_bytes;  // the image's own part of a batch workspace (index entries, LL buffers)
    Clock::time_point submitted;
};

dwt2::serve::Item item_of(const Pending &p)
{
    const uintptr_t s0 = (uintptr_t)p.r.src, d0 = (uintptr_t)p.r.dst;
    dwt2::serve::Item it{s0, s0 + span_bytes(p.r.src_pitch, p.r.width, p.r.height), d0,
                         d0 + span_bytes(p.r.dst_pitch, p.r.width, p.r.height),
                         p.r.inverse, p.r.levels, p.ll_bytes, 0};
    it.footprint = dwt2::serve::footprint_of(it);
    return it;
}

struct Flight {
    hipEvent_t ev = nullptr;
    std::vector<unsigned long long> tickets;
    std::vector<Clock::time_point> submitted;
    std::vector<int> status;
    Clock::time_point launched;
    size_t off = 0, bytes = 0;
    size_t footprint = 0;  // input + output + LL bytes of its requests
};

size_t table_bytes(int count, int lmax) { return dwt2::batch_table_bytes(count, lmax); }

}  // namespace

struct dwt2_server {
    dwt2_options opt{};
    int max_batch = 256, max_inflight = 2;
    size_t footprint_cap = SIZE_MAX;  // bytes; SIZE_MAX: no cap
    size_t in_flight_footprint = 0;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;              // the inverse group's stream
    hipEvent_t fork = nullptr, join = nullptr;
    int device = 0;

    std::mutex m;
    std::condition_variable cv_sched, cv_compl, cv_done;
    std::deque<Pending> pending;
    std::deque<Flight> inflight;
    std::unordered_map<unsigned long long, dwt2_completion> done;
    std::unordered_map<unsigned long long, bool> outstanding;  // submitted, not yet waited for
    Arena space{0};
    std::vector<hipEvent_t> events;
    unsigned long long next_ticket = 1, retired = 0;
    bool stopping = false, sched_exited = false;
    std::thread sched, compl_;

    void schedule();
    void complete();
};

void dwt2_server::schedule()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(m);
    for (;;) {
        cv_sched.wait(lk, [&] {
            return (stopping && pending.empty()) ||
                   (!pending.empty() && (int)inflight.size() < max_inflight);
        });
        if (pending.empty()) break;

        // Take the longest admissible prefix of the pending queue.
        Group g[2];
        size_t fp = 0;
        auto item = [&](size_t i) { return item_of(pending[i]); };
        const size_t n = dwt2::serve::next_batch(item, pending.size(), max_batch, space,
                                                 footprint_cap - in_flight_footprint, table_bytes, g, &fp);
        if (n == 0) {
            if (inflight.empty()) {
                // Unreachable: submission rejects a request larger than the
                // whole arena or the footprint cap, and with nothing in
                // flight both are free.
                const Pending p = pending.front();
                pending.pop_front();
                done[p.ticket] = {DWT2_E_WORKSPACE, 0.0, us_between(p.submitted, Clock::now())};
                cv_done.notify_all();
                continue;
            }
            // The head does not fit the free arena or the footprint budget:
            // wait for a batch to retire.
            const unsigned long long seen = retired;
            cv_sched.wait(lk, [&] { return retired != seen; });
            continue;
        }
        Flight f;
        f.bytes = group_bytes(g[0], table_bytes) + group_bytes(g[1], table_bytes);
        f.off = space.alloc(f.bytes);
        f.footprint = fp;
        in_flight_footprint += fp;
        std::vector<Pending> take(pending.begin(), pending.begin() + n);
        pending.erase(pending.begin(), pending.begin() + n);
        if (!events.empty()) {
            f.ev = events.back();
            events.pop_back();
        }
        lk.unlock();

        std::vector<dwt2_image> img[2];
        std::vector<size_t> idx[2];
        for (size_t i = 0; i < take.size(); i++) {
            const dwt2_request &r = take[i].r;
            const int d = r.inverse ? 1 : 0;
            img[d].push_back({r.wavelet, r.levels, r.width, r.height, r.src, r.src_pitch, r.dst,
                              r.dst_pitch});
            idx[d].push_back(i);
        }
        f.tickets.resize(take.size());
        f.submitted.resize(take.size());
        f.status.assign(take.size(), DWT2_OK);
        for (size_t i = 0; i < take.size(); i++) {
            f.tickets[i] = take[i].ticket;
            f.submitted[i] = take[i].submitted;
        }
        f.launched = Clock::now();
        char *ws = arena + f.off;
        const bool both = !img[0].empty() && !img[1].empty();
        hipError_t e = hipSuccess;
        if (both) {  // fork: the side stream starts after the caller's earlier work
            e = hipEventRecord(fork, stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
        }
        for (int d = 0; d < 2; d++) {
            if (img[d].empty()) continue;
            const size_t b = group_bytes(g[d], table_bytes);
            const hipStream_t st_d = both && d ? side : stream;
            const int st = e != hipSuccess ? DWT2_E_HIP
                           : d ? dwt2_inverse_batch(img[d].data(), (int)img[d].size(),
                                                    DWT2_EXT_WHOLE_SYMMETRIC, &opt, ws, b, st_d)
                               : dwt2_forward_batch(img[d].data(), (int)img[d].size(),
                                                    DWT2_EXT_WHOLE_SYMMETRIC, &opt, ws, b, st_d);
            for (size_t i : idx[d]) f.status[i] = st;
            ws += b;
        }
        if (both && e == hipSuccess) {  // join: the caller's stream waits for the side stream
            e = hipEventRecord(join, side);
            if (e == hipSuccess) e = hipStreamWaitEvent(stream, join, 0);
            if (e != hipSuccess)
                for (int &st : f.status)
                    if (st == DWT2_OK) st = DWT2_E_HIP;
        }
        if (!f.ev && hipEventCreateWithFlags(&f.ev, hipEventDisableTiming) != hipSuccess)
            f.ev = nullptr;
        if (f.ev && hipEventRecord(f.ev, stream) != hipSuccess) {
            for (int &st : f.status)
                if (st == DWT2_OK) st = DWT2_E_HIP;
        }
        lk.lock();
        inflight.push_back(std::move(f));
        cv_compl.notify_one();
    }
    sched_exited = true;
    cv_compl.notify_one();
}

void dwt2_server::complete()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(m);
    for (;;) {
        cv_compl.wait(lk, [&] { return !inflight.empty() || sched_exited; });
        if (inflight.empty()) break;
        hipEvent_t ev = inflight.front().ev;
        lk.unlock();
        // No event (creation failed): fall back to the stream itself.
        const hipError_t e = ev ? hipEventSynchronize(ev) : hipStreamSynchronize(stream);
        const Clock::time_point now = Clock::now();
        lk.lock();
        Flight f = std::move(inflight.front());
        inflight.pop_front();
        for (size_t i = 0; i < f.tickets.size(); i++) {
            dwt2_completion c;
            c.status = f.status[i] != DWT2_OK ? f.status[i] : (e == hipSuccess ? DWT2_OK : DWT2_E_HIP);
            c.queue_us = us_between(f.submitted[i], f.launched);
            c.latency_us = us_between(f.submitted[i], now);
            done[f.tickets[i]] = c;
        }
        space.release(f.off, f.bytes);
        in_flight_footprint -= f.footprint;
        if (f.ev) events.push_back(f.ev);
        retired++;
        cv_done.notify_all();
        cv_sched.notify_one();
    }
}

namespace {

int request_footprint(const dwt2_server *s, const dwt2_request *r, size_t *ll_bytes)
{
    if (!r || (r->inverse != 0 && r->inverse != 1)) return DWT2_E_ARG;
    const dwt2_image im = {r->wavelet, r->levels, r->width, r->height, r->src, r->src_pitch,
                           r->dst, r->dst_pitch};
    size_t one = 0;
    const int st = dwt2_batch_workspace_bytes(&im, 1, &s->opt, &one);
    if (st != DWT2_OK) return st;
    // The request's own part of any batch workspace (its tile-image index
    // entries and LL buffers, each rounded up to 256 bytes, so the parts of a
    // batch's requests add up to at least what the batch lays out).
    *ll_bytes = one - dwt2::batch_table_bytes(1, r->levels);
    const uintptr_t s0 = (uintptr_t)r->src, d0 = (uintptr_t)r->dst, a0 = (uintptr_t)s->arena;
    const uintptr_t s1 = s0 + span_bytes(r->src_pitch, r->width, r->height);
    const uintptr_t d1 = d0 + span_bytes(r->dst_pitch, r->width, r->height);
    const uintptr_t a1 = a0 + s->arena_bytes;
    if ((s0 < d1 && d0 < s1) || (s0 < a1 && a0 < s1) || (d0 < a1 && a0 < d1)) return DWT2_E_ALIAS;
    if (one > s->arena_bytes) return DWT2_E_WORKSPACE;
    if ((s1 - s0) + (d1 - d0) + *ll_bytes > s->footprint_cap) return DWT2_E_WORKSPACE;
    return DWT2_OK;
}

}  // namespace

DWT2_EXPORT int dwt2_server_create(const dwt2_options *opt, const dwt2_server_config *cfg,
                                   void *arena, size_t arena_bytes, hipStream_t stream,
                                   dwt2_server **out)
{
    if (!out) return DWT2_E_ARG;
    *out = nullptr;
    dwt2_options o = {};
    if (opt) o = *opt;
    for (int r : o.reserved)
        if (r) return DWT2_E_ARG;
    if (o.scheme != DWT2_SCHEME_AUTO && o.scheme != DWT2_SCHEME_MONOLITHIC_STAR)
        return DWT2_E_UNSUPPORTED;
    // batches run at their own height, double-buffered
    if (o.tile_rows != 0 || o.lds_buffers != 0 || o.tile_order != 0 || o.fuse_tail != 0)
        return DWT2_E_UNSUPPORTED;
    if (o.norm != DWT2_NORM_UNIT_DC && o.norm != DWT2_NORM_PAPER) return DWT2_E_UNSUPPORTED;
    if (o.arithmetic < DWT2_ARITH_AUTO || o.arithmetic > DWT2_ARITH_FP64) return DWT2_E_UNSUPPORTED;
    int max_batch = 256, max_inflight = 2;
    size_t footprint_cap = SIZE_MAX;
    if (cfg) {
        for (int r : cfg->reserved)
            if (r) return DWT2_E_ARG;
        if (cfg->max_batch < 0 || cfg->max_batch > DWT2_BATCH_MAX || cfg->max_inflight < 0 ||
            cfg->max_footprint_mib < 0)
            return DWT2_E_ARG;
        if (cfg->max_batch) max_batch = cfg->max_batch;
        if (cfg->max_inflight) max_inflight = cfg->max_inflight;
        if (cfg->max_footprint_mib) footprint_cap = (size_t)cfg->max_footprint_mib << 20;
    }
    if (!arena || arena_bytes < kAlign) return DWT2_E_WORKSPACE;
    if ((uintptr_t)arena & (kAlign - 1)) return DWT2_E_ARG;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return DWT2_E_HIP;

    dwt2_server *s = new dwt2_server;
    s->opt = o;
    s->max_batch = max_batch;
    s->max_inflight = max_inflight;
    s->footprint_cap = footprint_cap;
    s->arena = (char *)arena;
    s->arena_bytes = arena_bytes / kAlign * kAlign;
    s->space = Arena(s->arena_bytes);
    s->stream = stream;
    s->device = device;
    if (hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&s->join, hipEventDisableTiming) != hipSuccess) {
        if (s->join) (void)hipEventDestroy(s->join);
        if (s->fork) (void)hipEventDestroy(s->fork);
        if (s->side) (void)hipStreamDestroy(s->side);
        delete s;
        return DWT2_E_HIP;
    }
    s->sched = std::thread([s] { s->schedule(); });
    s->compl_ = std::thread([s] { s->complete(); });
    *out = s;
    return DWT2_OK;
}

DWT2_EXPORT int dwt2_server_submit(dwt2_server *s, const dwt2_request *r, unsigned long long *ticket)
{
    if (!s || !ticket) return DWT2_E_ARG;
    size_t ll = 0;
    const int st = request_footprint(s, r, &ll);
    if (st != DWT2_OK) return st;
    std::lock_guard<std::mutex> lk(s->m);
    if (s->stopping) return DWT2_E_STATE;
    const unsigned long long t = s->next_ticket++;
    s->pending.push_back({t, *r, ll, Clock::now()});
    s->outstanding[t] = true;
    *ticket = t;
    s->cv_sched.notify_one();
    return DWT2_OK;
}

DWT2_EXPORT int dwt2_server_wait(dwt2_server *s, unsigned long long ticket, dwt2_completion *out)
{
    if (!s) return DWT2_E_ARG;
    std::unique_lock<std::mutex> lk(s->m);
    if (!s->outstanding.count(ticket)) return DWT2_E_STATE;
    s->cv_done.wait(lk, [&] { return s->done.count(ticket) > 0; });
    const dwt2_completion c = s->done[ticket];
    s->done.erase(ticket);
    s->outstanding.erase(ticket);
    if (out) *out = c;
    return c.status;
}

DWT2_EXPORT int dwt2_server_replay(dwt2_server *s, const dwt2_request *reqs, const double *arrival_us,
                                   int count, dwt2_completion *out)
{
    if (!s || count < 0 || (count > 0 && (!reqs || !arrival_us || !out))) return DWT2_E_ARG;
    for (int i = 1; i < count; i++)
        if (arrival_us[i] < arrival_us[i - 1]) return DWT2_E_ARG;
    std::vector<unsigned long long> tickets(count, 0);
    int first_err = DWT2_OK, submitted = 0;
    const Clock::time_point t0 = Clock::now();
    for (; submitted < count; submitted++) {
        const Clock::time_point due =
            t0 + std::chrono::duration_cast<Clock::duration>(
                     std::chrono::duration<double, std::micro>(arrival_us[submitted]));
        while (Clock::now() < due) {
        }
        const int st = dwt2_server_submit(s, &reqs[submitted], &tickets[submitted]);
        if (st != DWT2_OK) {
            first_err = st;
            break;
        }
    }
    for (int i = 0; i < count; i++) {
        if (i < submitted) {
            dwt2_server_wait(s, tickets[i], &out[i]);
        } else {
            out[i].status = i == submitted ? first_err : DWT2_E_STATE;
            out[i].queue_us = out[i].latency_us = 0.0;
        }
    }
    return first_err;
}

DWT2_EXPORT int dwt2_server_destroy(dwt2_server *s)
{
    if (!s) return DWT2_E_ARG;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stopping = true;
    }
    s->cv_sched.notify_all();
    s->sched.join();
    s->compl_.join();
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    // every batch joined the side stream into the caller's stream before its
    // completion event, and the completer has waited for all of them
    (void)hipEventDestroy(s->join);
    (void)hipEventDestroy(s->fork);
    (void)hipStreamDestroy(s->side);
    delete s;
    return DWT2_OK;
}
