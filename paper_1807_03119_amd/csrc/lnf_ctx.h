// Context state behind an lnf_handle, and host helpers shared by the C-ABI
// translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "lnf.h"
#include "lnf_internal.h"

namespace lnf {

struct BatchState;  // batch.hip: job-table staging slots of lnf_filter_batch
using TuneKey = uint64_t;
TuneKey tune_key(int rule, int dtype, int radius, Geom g);

}  // namespace lnf

struct lnf_ctx {
    int device = 0;
    int rule = LNF_MEAN9;
    uint32_t gate = 0;
    uint32_t geom = 0;      // LNF_GEOM_* bits (0: cubes at offset r)
    mutable std::mutex mu;  // guards `tuned`
    std::unordered_map<lnf::TuneKey, lnf::TileCfg> tuned;
    void* dev_state = nullptr;  // library-internal device memory (see ctx_init_device_state)
    lnf::BatchState* batch = nullptr;  // job-table slots of lnf_filter_batch (lnf_create)
    std::mutex otsu_mu;                 // guards the Otsu scratch below
    uint64_t* otsu_dev = nullptr;       // 65536 histogram counters (lnf_filter_otsu)
    uint64_t* otsu_host = nullptr;      // pinned copy read by the host
    int64_t* entropy_dev = nullptr;     // 65536 fixed-point level weights (lnf_filter_entropy)
};

namespace lnf {

class DeviceGuard {
public:
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
    bool ok() const { return ok_; }

private:
    int prev_ = -1;
    bool ok_ = true;
    bool switched_ = false;
};

int check_volume_args(const lnf_ctx* h, const void* vol, const int64_t dims[3], int dtype,
                      int radius, const void* out, Geom* g, size_t* bytes);
int check_device_range(const void* p, size_t bytes, int device);
TileCfg ctx_tile(const lnf_ctx* h, int rule, int dtype, int radius, Geom g);
hipError_t launch_rule(int rule, uint32_t geom, const void* in, void* out, int dtype, int r,
                       Geom g, uint32_t gate, TileCfg cfg, hipStream_t s,
                       TileCfg* plan = nullptr);

// Batch path (batch.hip).
int validate_jobs(const lnf_ctx* h, const lnf_job* jobs, int n, std::vector<Geom>* geoms);
int batch_state_init(lnf_ctx* h);  // the job-table slots (freed by batch_state_free)
void batch_state_free(lnf_ctx* h);
void otsu_scratch_free(lnf_ctx* h);
void entropy_scratch_free(lnf_ctx* h);
// Histogram of n voxels into hist (cleared first), asynchronous on s (histogram.hip).
hipError_t launch_histogram(const void* vol, size_t n, int dtype, uint64_t* hist, hipStream_t s);

// Allocate / release the context's internal device memory.
int ctx_init_device_state(lnf_ctx* c);
void ctx_free_device_state(lnf_ctx* c);

}  // namespace lnf
