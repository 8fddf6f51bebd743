// cube_tune.hip -- the autotuner of the single-box pass.
//
// It times candidate launch shapes (threads per block, float4 loads per
// pipelined tile, LDS histogram copies, blocks per CU, the static or a
// dynamic partition with its chunk size, and for histograms the plain or the
// hot-bin LDS form) of one pass kind on
// the caller's own data with HIP events, and keeps the fastest shape per
// (pass kind, histogram-size class, box-size class) in a table that the
// launch planner consults when no explicit shape is set.  The table can be
// saved to and loaded from a small JSON file, keyed by the GPU architecture.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "cube_internal.h"

namespace cube {

namespace {

struct TuneKey {
    int kind, bins_log2, size_log2;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(kind, bins_log2, size_log2) < std::tie(o.kind, o.bins_log2, o.size_log2);
    }
};

std::mutex g_tmu;
std::map<TuneKey, TunedShape> g_table;
bool g_have_batch_rule = false;
BatchRule g_batch_rule = DEFAULT_BATCH_RULE;

int ilog2_ceil(uint64_t v)
{
    int k = 0;
    while (k < 63 && ((uint64_t)1 << k) < v) ++k;
    return k;
}

TuneKey key_of(int kind, int nbins, uint64_t voxels)
{
    return TuneKey{kind, kind == CUBE_Q_STATS ? 0 : ilog2_ceil((uint64_t)nbins),
                   ilog2_ceil(voxels < 1 ? 1 : voxels)};
}

}  // namespace

bool tuned_batch_rule(BatchRule *out)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_have_batch_rule) return false;
    *out = g_batch_rule;
    return true;
}

void set_tuned_batch_rule(const BatchRule &r)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    g_batch_rule = r;
    g_have_batch_rule = true;
}

bool batch_rule_ok(const BatchRule &r)
{
    return (r.threads == 256 || r.threads == 512 || r.threads == 1024) &&
           (r.unroll == 2 || r.unroll == 4) && r.floor_log2 >= 12 &&
           r.floor_log2 <= 30 && r.cap_log2 >= r.floor_log2 && r.cap_log2 <= 30 &&
           r.tiles_log2 >= 0 && r.tiles_log2 <= 20 && r.lds_kib >= 16 && r.lds_kib <= 160;
}

bool tuned_shape(int kind, int nbins, uint64_t voxels, TunedShape *out)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    auto it = g_table.find(key_of(kind, nbins, voxels));
    if (it == g_table.end()) return false;
    *out = it->second;
    return true;
}

}  // namespace cube

using namespace cube;

extern "C" {

int cube_autotune(const float *ptr, const int64_t *dims, int32_t kind, float lo, float hi,
                  int32_t nbins, int32_t reps, char *report, size_t report_cap)
{
    CUBE_GUARD_BEGIN
    if (kind != CUBE_Q_STATS && kind != CUBE_Q_HIST && kind != CUBE_Q_FUSED)
        return fail(CUBE_EINVAL, "autotune kinds: CUBE_Q_STATS, CUBE_Q_HIST, CUBE_Q_FUSED");
    if (reps < 1 || reps > 100) return fail(CUBE_EINVAL, "reps outside [1, 100]");
    Box box;
    int rc = check_box(ptr, dims, &box);
    if (!rc) rc = check_box_device(&box);
    if (rc) return rc;
    if (box.n == 0) return fail(CUBE_EINVAL, "nothing to tune on an empty box");
    HistRange r;
    if (kind != CUBE_Q_STATS && (rc = check_range(lo, hi, nbins, &r))) return rc;
    if (kind == CUBE_Q_STATS) nbins = 1;
    hipStream_t s = nullptr;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "tune stream");
    cube_stats_t *d_out = nullptr;
    unsigned long long *d_counts = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((e = hipMalloc(&d_out, sizeof(cube_stats_t))) != hipSuccess ||
        (e = hipMalloc(&d_counts, ((size_t)nbins + 3) * 8)) != hipSuccess ||
        (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        hipFree(d_out);
        hipFree(d_counts);
        hipStreamDestroy(s);
        return hip_fail(e, "tune buffers");
    }
    const int cus = cu_count();
    // Partitions: static, and dynamic with chunks of 2^18, 2^19, 2^20 voxels
    // (the dynamic pass exists for FP64MERGE moments only).
    const int part_c[] = {0, 18, 19, 20};
    const bool dyn_ok = accum_mode() == CUBE_ACCUM_FP64MERGE;
    const int hot_c[] = {0, 1};
    const int threads_c[] = {256, 512, 1024};
    const int unroll_c[] = {2, 4};
    const int copies_c[] = {8, 16, 32};
    const int bpc_c[] = {1, 2, 4, 8};
    struct Cand {
        TunedShape sh;
        float ms;
    };
    std::vector<Cand> cands;
    // Save the caller's explicit shape; each candidate is set explicitly.
    int prev_t, prev_b, prev_c, prev_u;
    get_launch(&prev_t, &prev_b, &prev_c, &prev_u);
    auto run_one = [&](void) -> int {
        switch (kind) {
        case CUBE_Q_STATS: return cube_stats_async(ptr, dims, d_out, s);
        case CUBE_Q_HIST: return cube_hist_async(ptr, dims, lo, hi, nbins,
                                                 (uint64_t *)d_counts, s);
        default: return cube_stats_hist_async(ptr, dims, lo, hi, nbins, d_out,
                                              (uint64_t *)d_counts, s);
        }
    };
    const int prev_hot = hot_override();
    const int prev_chunk = chunk_override();
    // Bring the shader clock up first: after idle it ramps over some tens of
    // milliseconds of sustained load, which would slow the first candidates.
    rc = CUBE_OK;
    for (int i = 0; i < 16 && !rc; ++i) rc = run_one();
    for (int part : part_c)
    for (int hot : hot_c)
    for (int t : threads_c)
        for (int u : unroll_c)
            for (int c : copies_c) {
                if (rc) break;
                if (part && (hot || !dyn_ok)) continue;
                if (kind == CUBE_Q_STATS && (c != copies_c[0] || hot)) continue;
                // The LDS histogram must fit one block (160 KiB); the hot-bin
                // form exists for LDS histograms only.
                if (kind != CUBE_Q_STATS && ((size_t)(nbins + 2) * c * 4 > 160 * 1024)) continue;
                if (hot && nbins > 32768) continue;
                set_hot_override(hot);
                set_chunk_override(part);
                for (int bpc : bpc_c) {
                    // A dynamic partition runs one resident wave of blocks.
                    if (part && bpc > 2) continue;
                    const int blocks = std::min(cus * bpc, 4096);
                    if ((rc = cube_set_launch(t, blocks, kind == CUBE_Q_STATS ? 0 : c, u))) break;
                    if ((rc = run_one())) break;  // warm-up
                    hipEventRecord(e0, s);
                    for (int i = 0; i < reps && !rc; ++i) rc = run_one();
                    hipEventRecord(e1, s);
                    if (rc) break;
                    if ((e = hipEventSynchronize(e1)) != hipSuccess) {
                        rc = hip_fail(e, "tune synchronize");
                        break;
                    }
                    float ms = 0.f;
                    hipEventElapsedTime(&ms, e0, e1);
                    Cand cd;
                    cd.sh.threads = t;
                    cd.sh.unroll = u;
                    cd.sh.copies = kind == CUBE_Q_STATS ? 0 : c;
                    cd.sh.blocks_per_cu = bpc;
                    cd.sh.hot = hot;
                    cd.sh.chunk_log2 = part;
                    cd.sh.ms = ms / reps;
                    cd.ms = ms / reps;
                    cands.push_back(cd);
                }
            }
    cube_set_launch(prev_t, prev_b, prev_c, prev_u);
    set_hot_override(prev_hot);
    set_chunk_override(prev_chunk);
    hipStreamSynchronize(s);
    release_ws(s);  // before the stream goes: its workspace is keyed by it
    hipFree(d_out);
    hipFree(d_counts);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipStreamDestroy(s);
    if (rc) return rc;
    if (cands.empty()) return fail(CUBE_EINVAL, "no launch shape fits these arguments");
    std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.ms < b.ms; });
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        g_table[key_of(kind, nbins, box.n)] = cands[0].sh;
    }
    if (report && report_cap) {
        std::string rep = "{\"best\": ";
        char buf[256];
        auto fmt = [&](const TunedShape &sh) {
            snprintf(buf, sizeof buf,
                     "{\"threads\": %d, \"unroll\": %d, \"copies\": %d, \"blocks_per_cu\": %d, "
                     "\"hot\": %d, \"chunk_log2\": %d, \"ms\": %.5f}",
                     sh.threads, sh.unroll, sh.copies, sh.blocks_per_cu, sh.hot, sh.chunk_log2,
                     sh.ms);
            return std::string(buf);
        };
        rep += fmt(cands[0].sh) + ", \"worst\": " + fmt(cands.back().sh);
        snprintf(buf, sizeof buf, ", \"candidates\": %zu}", cands.size());
        rep += buf;
        snprintf(report, report_cap, "%s", rep.c_str());
    }
    return CUBE_OK;
    CUBE_GUARD_END
}

int cube_tune_save(const char *path)
{
    CUBE_GUARD_BEGIN
    if (!path) return fail(CUBE_EINVAL, "path is NULL");
    FILE *f = fopen(path, "w");
    if (!f) return fail(CUBE_EINVAL, "cannot write %s", path);
    std::lock_guard<std::mutex> lk(g_tmu);
    fprintf(f, "{\"arch\": \"gfx950\", \"entries\": [");
    bool first = true;
    if (g_have_batch_rule) {
        // The batched launch's rule (one per table).
        fprintf(f,
                "\n  {\"kind\": %d, \"batch_threads\": %d, \"unroll\": %d, \"floor_log2\": %d, "
                "\"cap_log2\": %d, \"tiles_log2\": %d, \"lds_kib\": %d, \"ms\": %.5f}",
                CUBE_TUNE_BATCH, g_batch_rule.threads, g_batch_rule.unroll, g_batch_rule.floor_log2,
                g_batch_rule.cap_log2, g_batch_rule.tiles_log2, g_batch_rule.lds_kib,
                g_batch_rule.ms);
        first = false;
    }
    for (auto &kv : g_table) {
        fprintf(f,
                "%s\n  {\"kind\": %d, \"bins_log2\": %d, \"size_log2\": %d, \"threads\": %d, "
                "\"unroll\": %d, \"copies\": %d, \"blocks_per_cu\": %d, \"ms\": %.5f, "
                "\"hot\": %d, \"chunk_log2\": %d}",
                first ? "" : ",", kv.first.kind, kv.first.bins_log2, kv.first.size_log2,
                kv.second.threads, kv.second.unroll, kv.second.copies, kv.second.blocks_per_cu,
                kv.second.ms, kv.second.hot, kv.second.chunk_log2);
        first = false;
    }
    fprintf(f, "\n]}\n");
    fclose(f);
    return CUBE_OK;
    CUBE_GUARD_END
}

// Minimal reader for the format cube_tune_save writes: one entry per line.
int cube_tune_load(const char *path)
{
    CUBE_GUARD_BEGIN
    if (!path) return fail(CUBE_EINVAL, "path is NULL");
    FILE *f = fopen(path, "r");
    if (!f) return fail(CUBE_EINVAL, "cannot read %s", path);
    char line[512];
    int n = 0;
    bool arch_ok = false;
    std::map<TuneKey, TunedShape> t;
    bool have_rule = false;
    BatchRule rule = DEFAULT_BATCH_RULE;
    while (fgets(line, sizeof line, f)) {
        if (strstr(line, "\"arch\": \"gfx950\"")) arch_ok = true;
        const char *brace = strchr(line, '{');
        int bk;
        double bms;
        BatchRule r;
        if (brace && sscanf(brace,
                            "{\"kind\": %d, \"batch_threads\": %d, \"unroll\": %d, "
                            "\"floor_log2\": %d, \"cap_log2\": %d, \"tiles_log2\": %d, "
                            "\"lds_kib\": %d, \"ms\": %lf}",
                            &bk, &r.threads, &r.unroll, &r.floor_log2, &r.cap_log2,
                            &r.tiles_log2, &r.lds_kib, &bms) == 8) {
            if (bk != CUBE_TUNE_BATCH || !batch_rule_ok(r)) {
                fclose(f);
                return fail(CUBE_EINVAL, "%s: bad batch rule", path);
            }
            r.ms = (float)bms;
            rule = r;
            have_rule = true;
            ++n;
            continue;
        }
        int kind, bl, sl, th, un, co, bp, hot = 0, cl = 0;
        double ms;
        // "hot" and "chunk_log2" are optional (tables written before the
        // hot-bin form or the dynamic partition have none).
        const int got = sscanf(strchr(line, '{') ? strchr(line, '{') : line,
                               "{\"kind\": %d, \"bins_log2\": %d, \"size_log2\": %d, "
                               "\"threads\": %d, \"unroll\": %d, \"copies\": %d, "
                               "\"blocks_per_cu\": %d, \"ms\": %lf, \"hot\": %d, "
                               "\"chunk_log2\": %d}",
                               &kind, &bl, &sl, &th, &un, &co, &bp, &ms, &hot, &cl);
        if (got >= 8) {
            if ((th != 256 && th != 512 && th != 1024) || (un != 2 && un != 4) ||
                co < 0 || co > 32 || (co & (co - 1)) || bp < 1 || bp > 64 ||
                (hot != 0 && hot != 1) ||
                (cl != 0 && (cl < CUBE_CHUNK_LOG2_MIN || cl > CUBE_CHUNK_LOG2_MAX)) ||
                (cl != 0 && hot != 0)) {
                fclose(f);
                return fail(CUBE_EINVAL, "%s: bad entry", path);
            }
            TunedShape sh;
            sh.threads = th;
            sh.unroll = un;
            sh.copies = co;
            sh.blocks_per_cu = bp;
            sh.hot = hot;
            sh.chunk_log2 = cl;
            sh.ms = (float)ms;
            t[TuneKey{kind, bl, sl}] = sh;
            ++n;
        }
    }
    fclose(f);
    if (!arch_ok) return fail(CUBE_EINVAL, "%s: not a gfx950 tuning table", path);
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto &kv : t) g_table[kv.first] = kv.second;
    if (have_rule) {
        g_batch_rule = rule;
        g_have_batch_rule = true;
    }
    return n;
    CUBE_GUARD_END
}

void cube_tune_clear(void)
{
    CUBE_GUARD_BEGIN
    std::lock_guard<std::mutex> lk(g_tmu);
    g_table.clear();
    g_have_batch_rule = false;
    g_batch_rule = DEFAULT_BATCH_RULE;
    CUBE_GUARD_VOID_END
}

}  // extern "C"
