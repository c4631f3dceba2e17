// Open-loop load generator for the streaming request loop: Poisson block
// arrivals over many streams, block lengths uniform in [block_min,
// block_max], each stream at its own direction, changing now and then.  It
// drives the loop only through the public stream_* calls (a client of the
// library, like any serving front end) and reports throughput and the
// arrival-to-done latency distribution.
#include <time.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "hrir_internal.h"

namespace {

int64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

double pct(std::vector<int64_t>& v, double q) {
    if (v.empty()) return 0.0;
    const size_t i = std::min(v.size() - 1, (size_t)std::floor(q * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + (ptrdiff_t)i, v.end());
    return (double)v[i] * 1e-6;
}

}  // namespace

using hrir::fail;

extern "C" int stream_loadgen(hrir_server* srv, const stream_load* cfg, stream_load_stats* st) {
    hrir::clear_error();
    if (!srv || !cfg || !st || !cfg->signal) return fail(HRIR_EINVAL, "stream_loadgen: null pointer");
    if (cfg->n_streams < 1 || cfg->block_min < 1 || cfg->block_max < cfg->block_min || cfg->block_max > 4096 ||
        cfg->signal_len < cfg->block_max || cfg->n_filters < 2 || cfg->duration_s <= 0.0 || cfg->max_blocks < 1 ||
        cfg->submit_threads < 0 || cfg->submit_threads > 64)
        return fail(HRIR_EINVAL, "stream_loadgen: bad configuration");
    int64_t info[8];
    int rc = stream_info(srv, info);
    if (rc) return rc;
    const int64_t launches0 = info[0], eagain0 = info[3];
    const int64_t cap = cfg->max_blocks;
    std::vector<int64_t> arrival((size_t)cap), admit((size_t)cap, -1), lag((size_t)cap, -1), lat, lat_srv, collect;
    lat.reserve((size_t)cap);
    lat_srv.reserve((size_t)cap);
    collect.reserve((size_t)cap);
    // per submitting thread: its count of admitted blocks, on a cache line of
    // its own (threads do not share a counter or a line of the arrival and
    // admission arrays: thread t owns the tags [t * per, (t + 1) * per))
    struct alignas(64) Count {
        std::atomic<int64_t> n{0};
    };
    const int T = std::max(1, std::min(cfg->submit_threads > 0 ? cfg->submit_threads : 1, cfg->n_streams));
    const int64_t per = cap / T;
    std::vector<Count> sub_count((size_t)T);
    auto submitted = [&] {
        int64_t n = 0;
        for (const Count& c : sub_count) n += c.n.load(std::memory_order_acquire);
        return n;
    };
    std::atomic<bool> submit_done{false};
    std::atomic<int64_t> give_up_ns{INT64_MAX};      // set once submission ends
    std::atomic<int> poll_error{0};
    int64_t out_samples = 0, n_done = 0, t_last_done = 0, max_wait = 0, max_gpu = 0;

    std::thread poller([&] {
        std::vector<hrir_result> res(4096);
        for (;;) {
            const int n = stream_poll(srv, res.data(), (int32_t)res.size(), 1000);
            if (n < 0) {
                poll_error = n;
                return;
            }
            const int64_t t_got = now_ns();
            for (int i = 0; i < n; ++i) {
                const hrir_result& r = res[(size_t)i];
                lat.push_back(r.t_done_ns - arrival[(size_t)r.tag]);
                lat_srv.push_back(r.t_done_ns - r.t_submit_ns);
                collect.push_back(t_got - r.t_done_ns);
                max_wait = std::max(max_wait, r.t_launch_ns - r.t_submit_ns);
                max_gpu = std::max(max_gpu, r.t_done_ns - r.t_launch_ns);
                out_samples += 2 * (int64_t)r.n;
                t_last_done = std::max(t_last_done, r.t_done_ns);
            }
            n_done += n;
            if (submit_done && n_done >= submitted()) return;
            if (n == 0) {
                if (now_ns() > give_up_ns) {          // results stopped coming: report, do not wait forever
                    poll_error = HRIR_EDEVICE;
                    return;
                }
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            }
        }
    });

    // T submitting threads, each a Poisson process of rate / T over its own
    // range of streams
    const bool open_loop = cfg->rate_hz > 0.0;
    const int64_t t0 = now_ns();
    const int64_t t_stop = t0 + (int64_t)(cfg->duration_s * 1e9);
    std::atomic<int> sub_error{0};
    std::vector<int64_t> sent(T, 0);
    auto submitter = [&](int t) {
        std::mt19937_64 rng(cfg->seed + 0x9E3779B97F4A7C15ull * (uint64_t)(t + 1));
        // a contiguous range of streams per thread: neighbouring streams'
        // per-stream state is then written by one thread only
        const int s_begin = (int)((int64_t)cfg->n_streams * t / T);
        const int my_streams = (int)((int64_t)cfg->n_streams * (t + 1) / T) - s_begin;
        std::uniform_int_distribution<int> len_d(cfg->block_min, cfg->block_max);
        std::uniform_int_distribution<int> sid_d(0, my_streams - 1);
        std::uniform_int_distribution<int> dir_d(0, cfg->n_filters / 2 - 1);
        std::uniform_int_distribution<int64_t> off_d(0, cfg->signal_len - cfg->block_max);
        std::exponential_distribution<double> gap_d(open_loop ? cfg->rate_hz / T : 1.0);
        std::vector<int> dir((size_t)my_streams);
        for (int& d : dir) d = dir_d(rng);
        double t_next = (double)t0;
        int64_t j = 0;
        for (;;) {
            const int64_t tag = t * per + j;
            if (j >= per || poll_error != 0 || sub_error != 0) break;
            int64_t t_arr;
            if (open_loop) {
                t_next += gap_d(rng) * 1e9;
                t_arr = (int64_t)t_next;
                if (t_arr >= t_stop) break;
                for (int64_t tn; (tn = now_ns()) < t_arr;)
                    if (t_arr - tn > 200000) std::this_thread::sleep_for(std::chrono::microseconds(50));
            } else {
                t_arr = now_ns();
                if (t_arr >= t_stop) break;
            }
            const int ls = sid_d(rng);
            const int sid = s_begin + ls;
            if ((rng() & 15) == 0) dir[(size_t)ls] = dir_d(rng);    // a direction change every ~16 blocks
            const int len = len_d(rng);
            const float* blk = cfg->signal + off_d(rng);
            arrival[(size_t)tag] = t_arr;
            // how late the generator itself is: a block due at t_arr is first
            // offered to the server only now
            lag[(size_t)tag] = now_ns() - t_arr;
            int r;
            for (int tries = 0;; ++tries) {
                r = stream_submit(srv, sid, blk, len, 2 * dir[(size_t)ls], 2 * dir[(size_t)ls] + 1, (uint64_t)tag);
                if (r != HRIR_EAGAIN) break;
                // back off: retrying at full speed would hold up the
                // threads that free the room
                const int spins = 64 << std::min(tries, 5);
                for (int i = 0; i < spins; ++i) __builtin_ia32_pause();
            }
            if (r) {
                sub_error = r;
                break;
            }
            admit[(size_t)tag] = now_ns() - t_arr;
            ++j;
            sub_count[(size_t)t].n.store(j, std::memory_order_release);
        }
        sent[(size_t)t] = j;
    };
    std::vector<std::thread> subs;
    for (int t = 1; t < T; ++t) subs.emplace_back(submitter, t);
    submitter(0);
    for (auto& th : subs) th.join();
    const int64_t n = submitted();
    rc = sub_error.load();
    const int64_t t_sub_end = now_ns();
    give_up_ns = t_sub_end + 30000000000LL;
    submit_done = true;
    poller.join();
    if (rc) return fail(rc, "stream_loadgen: a submission failed");
    if (poll_error)
        return fail(poll_error, "stream_loadgen: %s", poll_error == HRIR_EDEVICE && n_done < submitted()
                                                          ? "results stopped arriving for 30 s"
                                                          : "poll failed");
    rc = stream_info(srv, info);
    if (rc) return rc;
    std::memset(st, 0, sizeof *st);
    st->blocks = n;
    st->out_samples = out_samples;
    st->eagain = info[3] - eagain0;
    st->launches = info[0] - launches0;
    st->offered_hz = open_loop ? cfg->rate_hz : 0.0;
    st->submit_s = (double)(t_sub_end - t0) * 1e-9;
    st->wall_s = (double)(std::max(t_last_done, t_sub_end) - t0) * 1e-9;
    st->achieved_hz = st->wall_s > 0 ? (double)n / st->wall_s : 0.0;
    st->out_samples_per_s = st->wall_s > 0 ? (double)out_samples / st->wall_s : 0.0;
    st->mean_batch = st->launches ? (double)n / (double)st->launches : 0.0;
    st->p50_ms = pct(lat, 0.50);
    st->p99_ms = pct(lat, 0.99);
    st->max_ms = pct(lat, 1.0);
    st->p50_server_ms = pct(lat_srv, 0.50);
    st->p99_server_ms = pct(lat_srv, 0.99);
    std::vector<int64_t> adm;
    adm.reserve((size_t)n);
    for (int64_t a : admit)
        if (a >= 0) adm.push_back(a);
    st->p99_admit_ms = pct(adm, 0.99);
    st->max_admit_ms = pct(adm, 1.0);
    adm.clear();
    for (int64_t a : lag)
        if (a >= 0) adm.push_back(a);
    st->p99_gen_lag_ms = pct(adm, 0.99);
    st->max_gen_lag_ms = pct(adm, 1.0);
    st->p99_collect_ms = pct(collect, 0.99);
    st->max_collect_ms = pct(collect, 1.0);
    st->max_wait_ms = (double)max_wait * 1e-6;
    st->max_launch_ms = (double)max_gpu * 1e-6;
    return HRIR_OK;
}
