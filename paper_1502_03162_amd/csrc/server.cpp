// Streaming request loop with continuous batching over the block renderer
// (Sec. IV-F: partitioned time-domain convolution, no added latency).
//
// Callers submit blocks of many streams at any time; the loop gathers what
// has arrived into a generation (at most one block per stream, since a
// stream's blocks must run in order through its history) and launches it as
// soon as fewer than kDepth generations are on the device, so blocks that
// arrive while others render join the next launch.  Generations live in a
// ring of G buffers (pinned host staging + device memory, sized from the HBM
// budget); a block is admitted into the oldest generation that can take it
// and is refused with HRIR_EAGAIN when none of the G buffers can.
//
// Per generation, on one of two HIP streams (alternating):
//   copy job table and inputs host -> device,
//   wait for the previous generation's kernel (stream histories),
//   block kernel (persistent grid from a HIP graph, or one workgroup per job),
//   copy outputs device -> host pinned memory, record the done event.
// Copies of one generation overlap the kernel of the other.  With
// STREAM_ZERO_COPY the ring lives in pinned, coherent host memory that the
// kernel reads and writes in place: a generation is the wait and the launch.
// A completion thread turns done events into results, handed out by
// stream_poll; it polls the done event with pauses, or with
// STREAM_SLEEPING_COMPLETION sleeps in the HIP runtime on a blocking-sync event.
//
// Admission takes no lock.  Each generation has one 64-bit reservation word
// (closed bit, epoch, jobs, output samples); a submission claims a job slot
// and its sample range with a compare-and-swap on it, fills them in, and
// marks its slot ready.  The loop thread launches a generation by setting
// its closed bit, which fixes its job count, and waits until that many slots
// are ready.  Only opening a new generation, finished generations and
// errors go through the server's mutex: the completion thread queues a
// finished generation, not its results, and stream_poll reads the results
// out of the generation's own tables.  A stream's
// blocks keep their order because its next block only goes into a later
// generation than its last one; submissions for one stream must therefore
// not overlap in time (those of different streams may).
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "block_internal.h"

using namespace hrir;

namespace {

constexpr int kDepth = 2;          // generations on the device at once
constexpr int kMaxGens = 8;
constexpr int kPersistentGrid = 1024;

int64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

enum GenState { kFree, kOpen, kLaunched, kDone, kHanded };

// Reservation word of a generation: bit 63 closed, bits 53..62 epoch (the
// generation's sequence number / ring size, mod 2^10, so that a submission
// that read a stale sequence number cannot reserve in a recycled buffer),
// bits 32..52 jobs, bits 0..31 output samples per ear.  A block's input sits
// at the same offset as its output samples (flush jobs leave input unused).
constexpr uint64_t kClosed = 1ull << 63;
constexpr int kEpochShift = 53;
constexpr uint64_t kEpochMask = 0x3ffull;
constexpr int kJobShift = 32;
constexpr uint64_t kJobMask = (1ull << 21) - 1;
constexpr uint64_t kOutMask = (1ull << 32) - 1;

inline uint64_t word_epoch(uint64_t w) { return (w >> kEpochShift) & kEpochMask; }
inline int word_jobs(uint64_t w) { return (int)((w >> kJobShift) & kJobMask); }
inline int64_t word_out(uint64_t w) { return (int64_t)(w & kOutMask); }

// Per job slot, beside the job table: what the result reports, and `ready`
// = generation sequence + 1 once the submission has filled the slot in.
struct Slot {
    uint64_t tag;
    int64_t t_submit;
    std::atomic<int64_t> ready{0};
    int64_t pad;
};

struct Gen {
    int64_t seq = -1;                      // set when opened, before the word is reset
    std::atomic<uint64_t> word{kClosed};
    GenState state = kFree;                // under the server mutex
    int n_jobs = 0, max_m = 0;             // fixed at launch
    bool failed = false;                   // its launch failed: no results
    int64_t out_used = 0;                  // output samples per ear, fixed at launch
    int64_t t_launch = 0, t_done = 0;
    // pinned host: h_hdr[0] = job count, then the job table; inputs; outputs
    int32_t* h_hdr = nullptr;
    BJob* h_jobs = nullptr;
    float* h_in = nullptr;
    float* h_out = nullptr;
    // device mirror
    int32_t* d_hdr = nullptr;
    BJob* d_jobs = nullptr;
    float* d_in = nullptr;
    float* d_out = nullptr;
    hipEvent_t ev_kernel = nullptr, ev_done = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::unique_ptr<Slot[]> slot;          // per job slot
    int next_result = 0;                   // results of this generation handed out so far
};

}  // namespace

struct hrir_server {
    hrir_streams* streams = nullptr;
    BlockShape sh{};
    int flags = 0;
    int cap_jobs = 0, n_gens = 0;
    int64_t cap_samples = 0;
    int tail = 0;
    hipStream_t st[2] = {nullptr, nullptr};
    std::unique_ptr<Gen[]> gens;
    std::vector<int64_t> last_seq;          // per stream: generation of its newest block (its submitter's)

    std::mutex mu;                          // opening generations, results, errors, thread hand-offs
    std::condition_variable cv_work;        // dispatcher: new jobs, a free device slot, close
    std::condition_variable cv_done;        // completer: a launch; pollers: results
    std::atomic<int64_t> head{0};           // oldest generation not yet free
    std::atomic<int64_t> tail_seq{0};       // one past the newest opened generation
    std::atomic<int64_t> next_launch{0};
    int64_t next_done = 0;
    int64_t enqueued = 0;                   // generations whose device work is fully enqueued
    std::deque<int64_t> done_gens;          // finished generations with results not yet all handed out
    std::atomic<bool> closing{false};
    bool dispatcher_exited = false;
    std::atomic<int> err_code{0};
    std::string err_msg;
    // statistics
    int64_t n_launches = 0, n_results = 0, n_samples = 0, max_batch = 0;
    std::atomic<int64_t> n_eagain{0};

    std::thread dispatcher, completer;

    Gen& gen(int64_t seq) { return gens[(size_t)(seq % n_gens)]; }
    uint64_t epoch(int64_t seq) const { return (uint64_t)(seq / n_gens) & kEpochMask; }
};

namespace {

void set_error(hrir_server* s, const char* where, hipError_t e) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->err_code) {
        s->err_msg = std::string(where) + ": " + hipGetErrorString(e);
        s->err_code = HRIR_EDEVICE;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
}

// Opens generation `seq` (its buffer is free) for submissions.  Lock held.
void open_gen(hrir_server* s, int64_t seq) {
    Gen& g = s->gen(seq);
    g.seq = seq;
    g.state = kOpen;
    g.n_jobs = 0;
    g.max_m = 0;
    g.out_used = 0;
    g.failed = false;
    g.next_result = 0;
    g.word.store(s->epoch(seq) << kEpochShift, std::memory_order_release);
}

// Releases generations whose results have all been handed out, in order.
// Lock held.
void release_handed(hrir_server* s) {
    int64_t h = s->head.load(std::memory_order_relaxed);
    while (h < s->tail_seq.load(std::memory_order_relaxed) && s->gen(h).state == kHanded) {
        s->gen(h).state = kFree;
        ++h;
    }
    s->head.store(h, std::memory_order_release);
}

// Takes the server lock for a short critical section: spin on try_lock for
// about a microsecond before blocking, so that threads that meet at the lock
// hand it over without sleeping in the kernel.
std::unique_lock<std::mutex> lock_short(std::mutex& mu) {
    for (int i = 0; i < 64; ++i) {
        if (mu.try_lock()) return std::unique_lock<std::mutex>(mu, std::adopt_lock);
        for (int j = 0; j < 16; ++j) __builtin_ia32_pause();
    }
    return std::unique_lock<std::mutex>(mu);
}

// Reserves a job slot and m output samples in generation q; returns the
// word before the reservation, or 0 with *ok false when q cannot take it
// (closed, recycled, or full).
uint64_t reserve(hrir_server* s, Gen& g, int64_t q, int m, bool* ok) {
    const uint64_t ep = s->epoch(q);
    uint64_t w = g.word.load(std::memory_order_acquire);
    for (;;) {
        if ((w & kClosed) || word_epoch(w) != ep || word_jobs(w) >= s->cap_jobs || word_out(w) + m > s->cap_samples) {
            *ok = false;
            return 0;
        }
        const uint64_t nw = w + (1ull << kJobShift) + (uint64_t)m;
        if (g.word.compare_exchange_weak(w, nw, std::memory_order_acq_rel, std::memory_order_acquire)) {
            *ok = true;
            return w;
        }
    }
}

// Wakes the loop thread when generation q has just become launchable (it
// is the next to launch, holds its first job and a device slot is free).
// Every other change that can make it launchable notifies on its own (a
// completion frees a slot; close; an error), so a submission that does not
// complete this condition wakes nobody: the loop thread is not woken once
// per block.  The mutex orders the notification against the loop thread's
// check of its wait condition.
void wake_dispatcher(hrir_server* s, int64_t q) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (q == s->next_launch.load(std::memory_order_relaxed) && s->next_launch - s->next_done < kDepth)
        s->cv_work.notify_one();
}

int enqueue_job(hrir_server* s, int32_t stream, const float* block, int32_t n, int32_t filt_l, int32_t filt_r,
                uint64_t tag, bool end, const char* fn) {
    const int m = end ? s->tail : n;
    if (s->err_code.load(std::memory_order_acquire)) {
        std::lock_guard<std::mutex> lk(s->mu);
        return fail(s->err_code, "%s: %s", fn, s->err_msg.c_str());
    }
    if (s->closing.load(std::memory_order_acquire)) return fail(HRIR_EINVAL, "%s: the server is closing", fn);
    // the oldest generation after this stream's last block that can take it
    int64_t q = std::max(s->next_launch.load(std::memory_order_acquire), s->last_seq[stream] + 1);
    for (;; ++q) {
        if (q >= s->head.load(std::memory_order_acquire) + s->n_gens) {
            s->n_eagain.fetch_add(1, std::memory_order_relaxed);
            return fail(HRIR_EAGAIN, "%s: no generation buffer has room (poll to release results)", fn);
        }
        if (q >= s->tail_seq.load(std::memory_order_acquire)) {
            // q is the next generation to open (q never passes tail_seq:
            // next_launch and every stream's last generation are below it)
            auto lk = lock_short(s->mu);
            const int64_t ts = s->tail_seq.load(std::memory_order_relaxed);
            if (q >= ts) {
                if (q != ts || q >= s->head.load(std::memory_order_relaxed) + s->n_gens || s->gen(q).state != kFree) {
                    s->n_eagain.fetch_add(1, std::memory_order_relaxed);
                    return fail(HRIR_EAGAIN, "%s: no generation buffer has room (poll to release results)", fn);
                }
                open_gen(s, q);
                s->tail_seq.store(q + 1, std::memory_order_release);
            }
        }
        Gen& g = s->gen(q);
        bool ok = false;
        const uint64_t w = reserve(s, g, q, m, &ok);
        if (!ok) continue;
        // the slot is ours: fill it in, then mark it ready
        const int i = word_jobs(w);
        const int64_t off = word_out(w);
        g.h_jobs[i] = BJob{stream, end ? 0 : n, filt_l, filt_r, end ? (kJobFlush | kJobReset) : 0, 0, off, 2 * off};
        if (!end) std::memcpy(g.h_in + off, block, sizeof(float) * (size_t)n);
        Slot& sl = g.slot[(size_t)i];
        sl.tag = tag;
        sl.t_submit = now_ns();
        s->last_seq[stream] = g.seq;        // stable: g cannot launch before its slot is ready
        sl.ready.store(g.seq + 1, std::memory_order_release);
        if (i == 0) wake_dispatcher(s, g.seq);
        return HRIR_OK;
    }
}

// Enqueues generation g on HIP stream `st`; `prev` is the previous
// generation's kernel event (null for the first).
hipError_t launch_gen(hrir_server* s, Gen& g, hipStream_t st, hipEvent_t prev) {
    *g.h_hdr = g.n_jobs;
    const bool zc = (s->flags & STREAM_ZERO_COPY) != 0;     // the kernel reads the host tables in place
    hipError_t e = hipSuccess;
    if (!zc) e = hipMemcpyAsync(g.d_hdr, g.h_hdr, 64 + sizeof(BJob) * (size_t)g.n_jobs, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && g.out_used && !zc)      // inputs sit at their jobs' output offsets
        e = hipMemcpyAsync(g.d_in, g.h_in, sizeof(float) * (size_t)g.out_used, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && prev) e = hipStreamWaitEvent(st, prev, 0);
    if (e == hipSuccess) {
        if (g.exec)
            e = hipGraphLaunch(g.exec, st);
        else
            e = block_enqueue(s->streams, g.d_in, g.d_jobs, nullptr, g.n_jobs, g.n_jobs, g.max_m, g.d_out, st);
    }
    if (e == hipSuccess) e = hipEventRecord(g.ev_kernel, st);
    if (e == hipSuccess && !zc)
        e = hipMemcpyAsync(g.h_out, g.d_out, sizeof(float) * 2 * (size_t)g.out_used, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(g.ev_done, st);
    return e;
}

void dispatcher_main(hrir_server* s) {
    (void)hipSetDevice(s->sh.device);
    hipEvent_t prev = nullptr;
    // a generation has jobs once a submission has reserved a slot in it
    auto has_jobs = [&](int64_t q) {
        return q < s->tail_seq.load(std::memory_order_acquire) &&
               word_jobs(s->gen(q).word.load(std::memory_order_acquire)) > 0;
    };
    for (;;) {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_work.wait(lk, [&] {
            if (s->err_code) return true;
            const bool ready = has_jobs(s->next_launch);
            if (s->closing && !ready) return true;
            return ready && s->next_launch - s->next_done < kDepth;
        });
        const bool ready = has_jobs(s->next_launch);
        if (s->err_code || (s->closing && !ready)) {
            s->dispatcher_exited = true;
            s->cv_done.notify_all();
            return;
        }
        const int64_t seq = s->next_launch.load(std::memory_order_relaxed);
        Gen& g = s->gen(seq);
        // close the generation: no reservation succeeds after this, so its
        // job count is fixed; later submissions go to the next generations
        const uint64_t w = g.word.fetch_or(kClosed, std::memory_order_acq_rel);
        s->next_launch.store(seq + 1, std::memory_order_release);
        g.state = kLaunched;
        s->n_launches++;
        lk.unlock();
        // wait for the submissions that hold a slot to finish filling it in
        const int n_jobs = word_jobs(w);
        for (int i = 0; i < n_jobs; ++i)
            for (int spins = 0; g.slot[(size_t)i].ready.load(std::memory_order_acquire) != seq + 1; ++spins) {
                if (spins < 256)
                    __builtin_ia32_pause();
                else
                    std::this_thread::yield();
            }
        g.n_jobs = n_jobs;
        g.out_used = word_out(w);
        int max_m = 0;
        for (int i = 0; i < n_jobs; ++i) max_m = std::max(max_m, block_job_len(s->sh, g.h_jobs[i]));
        g.max_m = max_m;
        g.t_launch = now_ns();
        // the generation no longer takes submissions: its tables are stable
        const hipError_t e = launch_gen(s, g, s->st[seq & 1], prev);
        prev = g.ev_kernel;
        if (e != hipSuccess) {
            set_error(s, "stream loop launch", e);
            std::lock_guard<std::mutex> lk2(s->mu);
            g.failed = true;
            s->enqueued = seq + 1;
            s->dispatcher_exited = true;
            s->cv_done.notify_all();
            return;
        }
        // only now is the done event recorded for this generation: before
        // this, querying it would see an earlier use of the buffer
        lk.lock();
        s->max_batch = std::max<int64_t>(s->max_batch, g.n_jobs);
        s->enqueued = seq + 1;
        s->cv_done.notify_all();
    }
}

void completer_main(hrir_server* s) {
    (void)hipSetDevice(s->sh.device);
    for (;;) {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->next_done < s->enqueued || s->dispatcher_exited || s->err_code; });
        if (s->next_done >= s->enqueued) {
            if (s->dispatcher_exited || s->err_code) return;
            continue;
        }
        const int64_t seq = s->next_done;
        Gen& g = s->gen(seq);
        const bool failed = g.failed;
        lk.unlock();
        hipError_t e = hipSuccess;
        if (!failed) {
            if (s->flags & STREAM_SLEEPING_COMPLETION) {
                e = hipEventSynchronize(g.ev_done);    // a blocking-sync event: the thread sleeps
            } else {
                while ((e = hipEventQuery(g.ev_done)) == hipErrorNotReady) {
                    // back off between queries: the loop thread's enqueues share the runtime
                    for (int i = 0; i < 64; ++i) __builtin_ia32_pause();
                }
            }
        }
        const int64_t t_done = now_ns();
        if (e != hipSuccess) {
            set_error(s, "stream loop completion", e);
            return;
        }
        lk.lock();
        g.t_done = t_done;
        g.next_result = 0;
        if (failed) {
            g.state = kHanded;
        } else {
            g.state = kDone;
            s->done_gens.push_back(seq);
            s->n_results += g.n_jobs;
            s->n_samples += g.out_used;
        }
        ++s->next_done;
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

void free_server(hrir_server* s) {
    for (int gi = 0; s->gens && gi < s->n_gens; ++gi) {
        Gen& g = s->gens[(size_t)gi];
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
        if (g.ev_kernel) (void)hipEventDestroy(g.ev_kernel);
        if (g.ev_done) (void)hipEventDestroy(g.ev_done);
        (void)hipHostFree(g.h_hdr);
        (void)hipHostFree(g.h_in);
        (void)hipHostFree(g.h_out);
        if (!(s->flags & STREAM_ZERO_COPY)) {      // else the d_ pointers alias the host buffers
            (void)hipFree(g.d_hdr);
            (void)hipFree(g.d_in);
            (void)hipFree(g.d_out);
        }
    }
    for (hipStream_t& x : s->st)
        if (x) (void)hipStreamDestroy(x);
    if (s->streams) block_streams_destroy(s->streams);
    delete s;
}

}  // namespace

extern "C" int stream_open(const hrir_plan* plan, int32_t max_streams, int64_t hbm_budget, int32_t flags,
                           hrir_server** out) {
    clear_error();
    if (!plan || !out) return fail(HRIR_EINVAL, "stream_open: null pointer");
    *out = nullptr;
    if (max_streams < 1 || max_streams > (1 << 20))
        return fail(HRIR_EINVAL, "stream_open: max_streams=%d outside [1, 2^20]", max_streams);
    if (flags & ~(STREAM_DIRECT_LAUNCH | STREAM_ZERO_COPY | STREAM_SLEEPING_COMPLETION))
        return fail(HRIR_EINVAL, "stream_open: unknown flags 0x%x", flags);
    if (hbm_budget < 0) return fail(HRIR_EINVAL, "stream_open: hbm_budget %lld < 0", (long long)hbm_budget);
    int32_t shp[3];
    int rc = spconv_plan_shape(plan, shp);
    if (rc) return rc;
    // device memory free before anything of this server is allocated: the
    // default budget is a quarter of it, and what the sizing below places on
    // the device must fit in it
    size_t dev_free = 0, dev_total = 0;
    const hipError_t me = hipMemGetInfo(&dev_free, &dev_total);
    if (me != hipSuccess) return fail(HRIR_EDEVICE, "stream_open: %s", hipGetErrorString(me));
    if (hbm_budget == 0) hbm_budget = (int64_t)(dev_free / 4);
    const int lf = shp[0], lg = shp[2];
    const int tail = lf + lg - 2;
    const int64_t min_cap = std::max(kBlockMax, tail);
    auto* s = new (std::nothrow) hrir_server;
    if (!s) return fail(HRIR_ENOMEM, "stream_open: out of host memory");
    rc = block_streams_create(plan, max_streams, &s->streams);
    if (rc) {
        delete s;
        return rc;
    }
    s->sh = block_shape(s->streams);
    // device bytes: histories, then per generation a header + job table,
    // inputs (4 B per sample) and two output ears (8 B per sample)
    const int64_t hist_bytes = (int64_t)max_streams * s->sh.hist_stride * 4;
    const int64_t fixed = 64 + 32LL * max_streams;
    auto per_gen = [&](int64_t cap) { return fixed + 12 * cap; };
    const int64_t avail = hbm_budget - hist_bytes;
    int64_t cap = std::max<int64_t>(min_cap, (int64_t)max_streams * 1024);
    int64_t n_gens = avail > 0 ? avail / per_gen(cap) : 0;
    if (n_gens > kMaxGens) n_gens = kMaxGens;
    for (int G = 3; n_gens < 3 && G >= 2; --G) {
        cap = (avail / G - fixed) / 12 / 64 * 64;
        if (cap >= min_cap) {
            n_gens = G;
            break;
        }
    }
    if (n_gens < 2 || cap < min_cap) {
        free_server(s);
        return fail(HRIR_EINVAL, "stream_open: hbm_budget %lld too small; at least %lld bytes are needed",
                    (long long)hbm_budget, (long long)(hist_bytes + 2 * per_gen(min_cap)));
    }
    // the histories are already allocated; the ring goes to the device
    // unless it lives in pinned host memory
    const int64_t dev_bytes = hist_bytes + ((flags & STREAM_ZERO_COPY) ? 0 : n_gens * per_gen(cap));
    if (dev_bytes > (int64_t)dev_free) {
        free_server(s);
        return fail(HRIR_ENOMEM, "stream_open: the server needs %lld bytes of device memory, %lld are free",
                    (long long)dev_bytes, (long long)dev_free);
    }

    s->flags = flags;
    s->cap_jobs = max_streams;
    s->cap_samples = std::min<int64_t>(cap, (int64_t)kOutMask);   // the reservation word's sample field
    s->n_gens = (int)n_gens;
    s->tail = tail;
    s->last_seq.assign(max_streams, -1);
    s->gens.reset(new (std::nothrow) Gen[(size_t)s->n_gens]);
    if (!s->gens) {
        s->n_gens = 0;
        free_server(s);
        return fail(HRIR_ENOMEM, "stream_open: out of host memory");
    }
    hipError_t e = hipSuccess;
    for (hipStream_t& x : s->st)
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
    const size_t hdr_bytes = 64 + sizeof(BJob) * (size_t)s->cap_jobs;
    const int max_m = (int)min_cap;
    const bool zc = (flags & STREAM_ZERO_COPY) != 0;
    const unsigned host_flags = zc ? (hipHostMallocMapped | hipHostMallocCoherent) : hipHostMallocDefault;
    auto device_view = [](void* h, void** d) { return hipHostGetDevicePointer(d, h, 0); };
    for (int gi = 0; gi < s->n_gens; ++gi) {
        Gen& g = s->gens[(size_t)gi];
        g.slot.reset(new (std::nothrow) Slot[(size_t)s->cap_jobs]);
        if (!g.slot) e = hipErrorOutOfMemory;
        if (e == hipSuccess) e = hipHostMalloc((void**)&g.h_hdr, hdr_bytes, host_flags);
        if (e == hipSuccess) e = hipHostMalloc((void**)&g.h_in, sizeof(float) * (size_t)cap, host_flags);
        if (e == hipSuccess) e = hipHostMalloc((void**)&g.h_out, sizeof(float) * 2 * (size_t)cap, host_flags);
        if (zc) {
            if (e == hipSuccess) e = device_view(g.h_hdr, (void**)&g.d_hdr);
            if (e == hipSuccess) e = device_view(g.h_in, (void**)&g.d_in);
            if (e == hipSuccess) e = device_view(g.h_out, (void**)&g.d_out);
        } else {
            if (e == hipSuccess) e = hipMalloc((void**)&g.d_hdr, hdr_bytes);
            if (e == hipSuccess) e = hipMalloc((void**)&g.d_in, sizeof(float) * (size_t)cap);
            if (e == hipSuccess) e = hipMalloc((void**)&g.d_out, sizeof(float) * 2 * (size_t)cap);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&g.ev_kernel, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&g.ev_done, hipEventDisableTiming | ((flags & STREAM_SLEEPING_COMPLETION)
                                                                                  ? hipEventBlockingSync
                                                                                  : 0));
        if (e != hipSuccess) break;
        g.h_jobs = reinterpret_cast<BJob*>(reinterpret_cast<char*>(g.h_hdr) + 64);
        g.d_jobs = reinterpret_cast<BJob*>(reinterpret_cast<char*>(g.d_hdr) + 64);
        if (!(flags & STREAM_DIRECT_LAUNCH)) {
            // persistent grid over the job table, count read from the header;
            // LDS sized for the longest job, so one graph serves every batch
            const int grid = std::min(kPersistentGrid, s->cap_jobs);
            e = hipStreamBeginCapture(s->st[0], hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const hipError_t el =
                    block_enqueue(s->streams, g.d_in, g.d_jobs, g.d_hdr, 0, grid, max_m, g.d_out, s->st[0]);
                e = hipStreamEndCapture(s->st[0], &g.graph);
                if (e == hipSuccess) e = el;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
            if (e != hipSuccess) break;
        }
    }
    if (e != hipSuccess) {
        free_server(s);
        return fail(e == hipErrorOutOfMemory ? HRIR_ENOMEM : HRIR_EDEVICE, "stream_open: %s", hipGetErrorString(e));
    }
    s->dispatcher = std::thread(dispatcher_main, s);
    s->completer = std::thread(completer_main, s);
    *out = s;
    return HRIR_OK;
}

extern "C" int stream_submit(hrir_server* s, int32_t stream_id, const float* host_block, int32_t n, int32_t filt_l,
                             int32_t filt_r, uint64_t tag) {
    clear_error();
    if (!s || !host_block) return fail(HRIR_EINVAL, "stream_submit: null pointer");
    if (stream_id < 0 || stream_id >= s->cap_jobs)
        return fail(HRIR_EINVAL, "stream_submit: stream %d outside [0, %d)", stream_id, s->cap_jobs);
    if (n < 1 || n > kBlockMax) return fail(HRIR_EINVAL, "stream_submit: n=%d outside [1, %d]", n, kBlockMax);
    if (filt_l < 0 || filt_l >= s->sh.n_filt || filt_r < 0 || filt_r >= s->sh.n_filt)
        return fail(HRIR_EINVAL, "stream_submit: filter (%d, %d) outside [0, %d)", filt_l, filt_r, s->sh.n_filt);
    return enqueue_job(s, stream_id, host_block, n, filt_l, filt_r, tag, false, "stream_submit");
}

extern "C" int stream_end(hrir_server* s, int32_t stream_id, int32_t filt_l, int32_t filt_r, uint64_t tag) {
    clear_error();
    if (!s) return fail(HRIR_EINVAL, "stream_end: null pointer");
    if (stream_id < 0 || stream_id >= s->cap_jobs)
        return fail(HRIR_EINVAL, "stream_end: stream %d outside [0, %d)", stream_id, s->cap_jobs);
    if (filt_l < 0 || filt_l >= s->sh.n_filt || filt_r < 0 || filt_r >= s->sh.n_filt)
        return fail(HRIR_EINVAL, "stream_end: filter (%d, %d) outside [0, %d)", filt_l, filt_r, s->sh.n_filt);
    return enqueue_job(s, stream_id, nullptr, 0, filt_l, filt_r, tag, true, "stream_end");
}

extern "C" int stream_poll(hrir_server* s, hrir_result* out, int32_t max, int32_t timeout_us) {
    clear_error();
    if (!s || (max > 0 && !out)) return fail(HRIR_EINVAL, "stream_poll: null pointer");
    if (max < 0) return fail(HRIR_EINVAL, "stream_poll: max=%d < 0", max);
    auto lk = lock_short(s->mu);
    // results handed out by the previous poll are no longer referenced
    release_handed(s);
    // wake on results or an error; never wait when nothing is queued or running
    auto pending = [&] { return !s->done_gens.empty() || s->err_code || s->next_done == s->tail_seq; };
    if (timeout_us < 0)
        s->cv_done.wait(lk, pending);
    else if (timeout_us > 0)
        s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), pending);
    if (s->done_gens.empty() && s->err_code) return fail(s->err_code, "stream_poll: %s", s->err_msg.c_str());
    int n = 0;
    while (n < max && !s->done_gens.empty()) {
        Gen& g = s->gen(s->done_gens.front());
        const int take = std::min(max - n, g.n_jobs - g.next_result);
        for (int i = g.next_result; i < g.next_result + take; ++i) {
            const BJob& j = g.h_jobs[i];
            const Slot& sl = g.slot[(size_t)i];
            hrir_result& r = out[n++];
            r = hrir_result{};
            r.tag = sl.tag;
            r.stream_id = j.slot;
            r.n = block_job_len(s->sh, j);
            r.out = g.h_out + j.out_off;
            r.t_submit_ns = sl.t_submit;
            r.t_launch_ns = g.t_launch;
            r.t_done_ns = g.t_done;
            r.flags = (j.flags & kJobFlush) ? STREAM_RESULT_TAIL : 0;
        }
        g.next_result += take;
        if (g.next_result == g.n_jobs) {
            g.state = kHanded;              // freed by the next poll: the results point into it
            s->done_gens.pop_front();
        }
    }
    return n;
}

extern "C" int stream_info(const hrir_server* s, int64_t* info8) {
    clear_error();
    if (!s || !info8) return fail(HRIR_EINVAL, "stream_info: null pointer");
    auto* m = const_cast<hrir_server*>(s);
    std::lock_guard<std::mutex> lk(m->mu);
    int64_t queued = 0;
    for (int64_t q = s->next_launch; q < s->tail_seq; ++q) queued += word_jobs(m->gen(q).word.load());
    info8[0] = s->n_launches;
    info8[1] = s->n_results;
    info8[2] = s->n_samples;
    info8[3] = s->n_eagain.load();
    info8[4] = s->max_batch;
    info8[5] = s->n_gens;
    info8[6] = s->cap_samples;
    info8[7] = queued;
    return HRIR_OK;
}

extern "C" void stream_close(hrir_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->closing.store(true, std::memory_order_release);
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    if (s->dispatcher.joinable()) s->dispatcher.join();
    if (s->completer.joinable()) s->completer.join();
    for (hipStream_t x : s->st)
        if (x) (void)hipStreamSynchronize(x);
    free_server(s);
}
