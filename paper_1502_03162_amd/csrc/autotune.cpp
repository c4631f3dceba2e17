// Launch-shape autotuner for spconv batches: times candidate (tile length,
// jobs per tile, persistent, workgroup size) shapes of one job list with HIP events and
// keeps the fastest, optionally cached in a JSON file keyed by the plan's
// (K, lf, lg) and a coarse shape class of the job list.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

#include "hrir_internal.h"

namespace {

struct Shape {
    int tile, group, flags;
    double ms;
};

std::string shape_class(const int64_t* src_len, int n_src, const spconv_job* jobs, int n_jobs, int k, int lf,
                        int lg) {
    double outs = 0.0;
    std::vector<int> per(n_src, 0);
    for (int j = 0; j < n_jobs; ++j) {
        outs += (double)(src_len[jobs[j].src] + lf + lg - 2);
        per[jobs[j].src]++;
    }
    int used = 0;
    for (int v : per) used += v > 0;
    const double jps = used ? (double)n_jobs / used : 0.0;
    char buf[160];
    std::snprintf(buf, sizeof buf, "K%d_lf%d_lg%d_out2^%d_jobs_per_src%d_srcs2^%d", k, lf, lg,
                  (int)std::lround(std::log2(std::max(outs, 1.0))), (int)std::lround(jps),
                  (int)std::lround(std::log2(std::max(used, 1))));
    return buf;
}

// Cache file: {"<class>": [tile, group, flags, ms], ...}
std::map<std::string, Shape> read_cache(const char* path) {
    std::map<std::string, Shape> m;
    std::ifstream in(path);
    if (!in) return m;
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string s = ss.str();
    size_t pos = 0;
    while ((pos = s.find('"', pos)) != std::string::npos) {
        const size_t end = s.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = s.substr(pos + 1, end - pos - 1);
        const size_t lb = s.find('[', end), rb = s.find(']', end);
        if (lb == std::string::npos || rb == std::string::npos) break;
        Shape sh{};
        if (std::sscanf(s.c_str() + lb, "[%d , %d , %d , %lf]", &sh.tile, &sh.group, &sh.flags, &sh.ms) == 4 ||
            std::sscanf(s.c_str() + lb, "[%d, %d, %d, %lf]", &sh.tile, &sh.group, &sh.flags, &sh.ms) == 4)
            m[key] = sh;
        pos = rb + 1;
    }
    return m;
}

void write_cache(const char* path, const std::map<std::string, Shape>& m) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : m)
        std::fprintf(f, "  \"%s\": [%d, %d, %d, %.17g]%s\n", kv.first.c_str(), kv.second.tile, kv.second.group,
                     kv.second.flags, kv.second.ms, ++i < m.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

}  // namespace

using hrir::fail;

extern "C" int spconv_plan_shape(const hrir_plan* plan, int32_t* lf_k_lg3);

extern "C" int spconv_autotune(const hrir_plan* plan, const float* d_src, int64_t src_elems, const int64_t* src_off,
                               const int64_t* src_len, int32_t n_src, const spconv_job* jobs, int32_t n_jobs,
                               float* d_out, int64_t out_elems, void* stream, const char* cache_path,
                               int32_t force_flags, int32_t* tile_out, int32_t* group_out, int32_t* flags_out,
                               double* ms_out) {
    hrir::clear_error();
    if (!plan || !tile_out || !group_out || !flags_out) return fail(HRIR_EINVAL, "spconv_autotune: null pointer");
    int32_t shp[3];
    int rc = spconv_plan_shape(plan, shp);
    if (rc) return rc;
    const int lf = shp[0], k = shp[1], lg = shp[2];
    if (force_flags & ~(SPCONV_PERSISTENT | SPCONV_LDS_GATHER))
        return fail(HRIR_EINVAL, "spconv_autotune: force_flags may hold PERSISTENT and LDS_GATHER only");
    const std::string key =
        shape_class(src_len, n_src, jobs, n_jobs, k, lf, lg) + "_flags" + std::to_string(force_flags);
    std::map<std::string, Shape> cache;
    if (cache_path) {
        cache = read_cache(cache_path);
        auto it = cache.find(key);
        if (it != cache.end()) {
            *tile_out = it->second.tile;
            *group_out = it->second.group;
            *flags_out = it->second.flags;
            if (ms_out) *ms_out = it->second.ms;
            return HRIR_OK;
        }
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(HRIR_EDEVICE, "spconv_autotune: event creation failed");
    Shape best{0, 0, 0, 1e300};
    const int tiles[] = {1024, 2048, 3072, 4096};
    const int groups[] = {0, 4, 8, 16};
    for (int tile : tiles)
        for (int group : groups)
            for (int pers : {0, SPCONV_PERSISTENT})
            for (int wg : {0, SPCONV_WG256}) {
                if ((force_flags & SPCONV_PERSISTENT) && !pers) continue;
                if (wg && (force_flags & SPCONV_LDS_GATHER)) continue;
                const int flags = force_flags | pers | wg;
                hrir_batch* b = nullptr;
                if (spconv_batch_create(plan, src_off, src_len, n_src, jobs, n_jobs, tile, group, flags, &b)) continue;
                float ms = 0.0f;
                bool ok = spconv_batch_render(b, d_src, src_elems, d_out, out_elems, stream) == HRIR_OK;
                ok = ok && hipEventRecord(e0, st) == hipSuccess;
                for (int r = 0; ok && r < 3; ++r)
                    ok = spconv_batch_render(b, d_src, src_elems, d_out, out_elems, stream) == HRIR_OK;
                ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                spconv_batch_destroy(b);
                if (!ok) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return fail(HRIR_EDEVICE, "spconv_autotune: timing run failed: %s", hrir::last_error());
                }
                if (ms / 3.0 < best.ms) best = Shape{tile, group, flags, ms / 3.0};
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best.tile == 0) return fail(HRIR_EINVAL, "spconv_autotune: no candidate shape is valid for this job list");
    *tile_out = best.tile;
    *group_out = best.group;
    *flags_out = best.flags;
    if (ms_out) *ms_out = best.ms;
    if (cache_path) {
        cache[key] = best;
        write_cache(cache_path, cache);
    }
    return HRIR_OK;
}
