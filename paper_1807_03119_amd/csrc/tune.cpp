// Autotuner: picks, per (rule, dtype, radius, volume-size class), the tile
// variant and z-strip depth with the shortest kernel time, measured with HIP
// events on the sample jobs themselves.  Results live in the context and can
// be saved to / loaded from a text file (LNF_TUNE_CACHE is loaded at create).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <vector>

#include "lnf.h"
#include "lnf_ctx.h"
#include "lnf_internal.h"

namespace lnf {
namespace {

constexpr int kTimedRuns = 3;

std::vector<int> zs_candidates(int nz)
{
    std::vector<int> c = {0};  // 0: the launcher's default depth
    for (int z : {16, 32, 64, 128, 256})
        if (z < nz) c.push_back(z);
    c.push_back(nz);  // whole depth: one strip per column
    std::sort(c.begin(), c.end());
    c.erase(std::unique(c.begin(), c.end()), c.end());
    return c;
}

}  // namespace
}  // namespace lnf

using namespace lnf;

extern "C" int lnf_tune(lnf_handle h, const lnf_job* sample, int n)
{
    if (!h) return LNF_EINVAL;
    DeviceGuard dg(h->device);
    if (!dg.ok()) return LNF_EHIP;
    std::vector<Geom> geoms;
    int rc = validate_jobs(h, sample, n, &geoms);
    if (rc) return rc;
    // the largest sample job of every key represents it
    std::map<TuneKey, int> rep;
    for (int i = 0; i < n; ++i) {
        const TuneKey k = tune_key(h->rule, sample[i].dtype, sample[i].radius, geoms[i]);
        auto it = rep.find(k);
        const double v = (double)geoms[i].nx * geoms[i].ny * geoms[i].nz;
        if (it == rep.end() ||
            v > (double)geoms[it->second].nx * geoms[it->second].ny * geoms[it->second].nz)
            rep[k] = i;
    }
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = LNF_EHIP;
    }
    const int nv = h->rule == LNF_MEAN9 ? mean9_variants() : minvar9_variants();
    for (auto it = rep.begin(); rc == LNF_OK && it != rep.end(); ++it) {
        const lnf_job& j = sample[it->second];
        const Geom g = geoms[it->second];
        float best = 1e30f;
        TileCfg best_cfg{-1, 0};
        for (int v = 0; v < nv && rc == LNF_OK; ++v) {
            for (int zs : zs_candidates(g.nz)) {
                const TileCfg cfg{v, zs};
                if (launch_rule(h->rule, h->geom, j.in, j.out, j.dtype, j.radius, g, h->gate, cfg, s) !=
                    hipSuccess) {
                    rc = LNF_EHIP;
                    break;
                }
                (void)hipEventRecord(e0, s);
                for (int t = 0; t < kTimedRuns; ++t)
                    (void)launch_rule(h->rule, h->geom, j.in, j.out, j.dtype, j.radius, g, h->gate, cfg,
                                      s);
                (void)hipEventRecord(e1, s);
                float ms = 0.f;
                if (hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    rc = LNF_EHIP;
                    break;
                }
                if (ms < best) {
                    best = ms;
                    best_cfg = cfg;
                }
            }
        }
        if (rc == LNF_OK) {
            std::lock_guard<std::mutex> lk(h->mu);
            h->tuned[it->first] = best_cfg;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    return rc;
}

extern "C" int lnf_tune_save(lnf_handle h, const char* path)
{
    if (!h || !path) return LNF_EINVAL;
    FILE* f = std::fopen(path, "w");
    if (!f) return LNF_EINVAL;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        std::fprintf(f, "# lnf tune cache: key variant zs\n");
        for (const auto& kv : h->tuned)
            std::fprintf(f, "%llu %d %d\n", (unsigned long long)kv.first, kv.second.variant,
                         kv.second.zs);
    }
    return std::fclose(f) == 0 ? LNF_OK : LNF_EINVAL;
}

extern "C" int lnf_tune_load(lnf_handle h, const char* path)
{
    if (!h || !path) return LNF_EINVAL;
    FILE* f = std::fopen(path, "r");
    if (!f) return LNF_EINVAL;
    char line[256];
    std::map<TuneKey, TileCfg> got;
    int rc = LNF_OK;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        unsigned long long key = 0;
        int v = 0, zs = 0;
        if (std::sscanf(line, "%llu %d %d", &key, &v, &zs) != 3 || zs < 0 || v < -1) {
            rc = LNF_EINVAL;
            break;
        }
        const int rule = (int)(key >> 48);
        const int nv = rule == LNF_MEAN9 ? mean9_variants() : minvar9_variants();
        if (v >= nv) {
            rc = LNF_EINVAL;
            break;
        }
        got[(TuneKey)key] = TileCfg{v, zs};
    }
    std::fclose(f);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(h->mu);
    for (const auto& kv : got) h->tuned[kv.first] = kv.second;
    return LNF_OK;
}
