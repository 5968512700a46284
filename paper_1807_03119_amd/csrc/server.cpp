// Request server with continuous batching (contract: include/lnf.h, "serving").
//
// One worker thread per server owns scheduling:
//   - admission: pending requests are admitted in arrival order while the
//     device footprint (resident volumes + outputs + cached free blocks) stays
//     under the cap; to make room it drops cached blocks, then evicts idle
//     resident volumes least-recently-used first;
//   - micro-batching: requests admitted in one pass, up to max_batch of them
//     and the voxel budget, become one lnf_filter_batch launch on the next
//     stream of the pool (after waiting on the upload events of its volumes),
//     so later batches overlap earlier ones;
//   - device queue bound: a pass launches only while fewer than two batches
//     are in flight or their voxels stay under twice the budget.  Requests
//     beyond that wait in the host queue, where they are batched with later
//     arrivals, instead of piling up on the streams, where concurrent
//     batches would share the device and all finish late;
//   - completion: per-batch events are polled; latency is measured from each
//     request's scheduled arrival time to the moment its completion is seen.
// Device memory comes from an arena: chunks are allocated on demand up to the
// cap and kept until the server ends, and volumes and outputs take ranges of
// them from a best-fit free list that merges neighbours.  Evicting a volume
// only returns its range, so the steady state never reaches hipFree, which
// would synchronise the whole device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lnf.h"
#include "lnf_ctx.h"
#include "lnf_internal.h"

namespace lnf {
namespace {

int64_t steady_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Device ranges for the server: host-side bookkeeping over chunks that are
// allocated once and freed only by release_all().  Ranges never span two
// chunks (each chunk is its own allocation).
class Arena {
public:
    static constexpr size_t kAlign = 64u << 10;  // range granularity
    static constexpr size_t kChunk = 4ull << 30;  // preferred chunk size

    static size_t round(size_t bytes) { return (bytes + kAlign - 1) / kAlign * kAlign; }
    size_t reserved() const { return reserved_; }  // device bytes held in chunks
    size_t used() const { return used_; }          // bytes in ranges handed out

    // Best-fit range of `bytes` (a multiple of kAlign) from free space, or null.
    void* take(size_t bytes)
    {
        auto it = by_size_.lower_bound(bytes);
        if (it == by_size_.end()) return nullptr;
        char* p = it->second;
        const size_t have = it->first;
        by_size_.erase(it);
        by_addr_.erase(p);
        if (have > bytes) insert(p + bytes, have - bytes);
        used_ += bytes;
        return p;
    }

    // Return a range; merges with free neighbours inside the same chunk.
    void give(void* ptr, size_t bytes)
    {
        char* p = static_cast<char*>(ptr);
        used_ -= bytes;
        const char* chunk_end = chunk_of(p);
        auto next = by_addr_.find(p + bytes);
        if (next != by_addr_.end() && p + bytes < chunk_end) {
            bytes += next->second;
            erase(next);
        }
        auto prev = by_addr_.lower_bound(p);
        if (prev != by_addr_.begin()) {
            --prev;
            if (prev->first + prev->second == p && chunk_of(prev->first) == chunk_end) {
                p = prev->first;
                bytes += prev->second;
                erase(prev);
            }
        }
        insert(p, bytes);
    }

    // Allocate a chunk of at least `bytes` without the held total passing
    // `limit`.  hipMalloc does not synchronise the device.
    int grow(size_t bytes, size_t limit)
    {
        if (reserved_ + bytes > limit) return LNF_EBUSY;
        size_t want = std::min(std::max(kChunk, bytes), limit - reserved_);
        void* p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            want = bytes;
            if (hipMalloc(&p, want) != hipSuccess) {
                (void)hipGetLastError();
                return LNF_ENOMEM;
            }
        }
        chunks_[static_cast<char*>(p)] = want;
        reserved_ += want;
        insert(static_cast<char*>(p), want);
        return LNF_OK;
    }

    void release_all()
    {
        for (auto& c : chunks_) (void)hipFree(c.first);
        chunks_.clear();
        by_addr_.clear();
        by_size_.clear();
        reserved_ = used_ = 0;
    }

private:
    const char* chunk_of(const char* p) const  // end of the chunk holding p
    {
        auto it = chunks_.upper_bound(const_cast<char*>(p));
        --it;
        return it->first + it->second;
    }
    void insert(char* p, size_t n)
    {
        by_addr_[p] = n;
        by_size_.emplace(n, p);
    }
    void erase(std::map<char*, size_t>::iterator it)
    {
        auto range = by_size_.equal_range(it->second);
        for (auto s = range.first; s != range.second; ++s)
            if (s->second == it->first) {
                by_size_.erase(s);
                break;
            }
        by_addr_.erase(it);
    }

    std::map<char*, size_t> chunks_;          // start -> size
    std::map<char*, size_t> by_addr_;         // free ranges: start -> size
    std::multimap<size_t, char*> by_size_;    // free ranges: size -> start
    size_t reserved_ = 0, used_ = 0;
};

struct Volume {
    void* dev = nullptr;
    size_t block = 0;  // bytes of its arena range
    int64_t dims[3] = {0, 0, 0};
    int dtype = 0;
    hipEvent_t ready = nullptr;  // upload complete
    int refs = 0;                // requests (pending or in flight) using it
    bool released = false;       // client dropped it: free once refs == 0
    std::list<uint64_t>::iterator lru;
};

enum ReqState { kPending = 0, kInFlight = 1, kDone = 2 };

struct Request {
    uint64_t vol = 0;
    int radius = 1;
    void* host_out = nullptr;
    int64_t arrival = 0;
    int state = kPending;
    int status = LNF_OK;
    void* out = nullptr;
    size_t block = 0;
    uint64_t voxels = 0;
};

struct Flight {
    std::vector<uint64_t> tickets;
    hipEvent_t done = nullptr;
    uint64_t voxels = 0;
};

}  // namespace

class Server {
public:
    Server(lnf_handle h, const lnf_server_options& o)
        : h_(h), o_(o), budget_((uint64_t)(o.batch_mvox > 0 ? o.batch_mvox : 32) << 20)
    {
    }

    int init()
    {
        DeviceGuard dg(h_->device);
        if (!dg.ok()) return LNF_EHIP;
        const int ns = o_.mode == LNF_SERVE_FIFO ? 1 : o_.n_streams;
        for (int i = 0; i < ns; ++i) {
            hipStream_t s;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return LNF_EHIP;
            streams_.push_back(s);
        }
        if (hipStreamCreateWithFlags(&upload_, hipStreamNonBlocking) != hipSuccess) return LNF_EHIP;
        worker_ = std::thread([this] { loop(); });
        return LNF_OK;
    }

    ~Server()
    {
        {
            std::unique_lock<std::mutex> lk(mu_);
            stop_ = true;
            for (uint64_t t : pending_) finish(t, LNF_ECANCELED, 0);
            pending_.clear();
        }
        cv_.notify_all();
        if (worker_.joinable()) worker_.join();
        DeviceGuard dg(h_->device);
        for (auto& kv : vols_) {
            if (kv.second.ready) {
                (void)hipEventSynchronize(kv.second.ready);
                (void)hipEventDestroy(kv.second.ready);
            }
        }
        for (hipStream_t s : streams_) (void)hipStreamSynchronize(s);
        if (upload_) (void)hipStreamSynchronize(upload_);
        arena_.release_all();
        for (hipEvent_t e : free_events_) (void)hipEventDestroy(e);
        for (hipStream_t s : streams_) (void)hipStreamDestroy(s);
        if (upload_) (void)hipStreamDestroy(upload_);
    }

    int put(const void* host, const int64_t dims[3], int dtype, const int64_t* pitch, uint64_t* id)
    {
        if (!host || !dims || !id || (dtype != LNF_U8 && dtype != LNF_U16)) return LNF_EINVAL;
        for (int i = 0; i < 3; ++i)
            if (dims[i] < 1 || dims[i] > INT32_MAX) return LNF_EINVAL;
        if (dims[0] * dims[1] > INT32_MAX) return LNF_EINVAL;
        if (pitch && (pitch[0] < dims[0] || pitch[1] < pitch[0] * dims[1])) return LNF_EINVAL;
        const size_t es = dtype == LNF_U8 ? 1 : 2;
        const size_t bytes = (size_t)dims[0] * dims[1] * dims[2] * es;
        DeviceGuard dg(h_->device);
        std::unique_lock<std::mutex> lk(mu_);
        Volume v;
        int rc = get_block(bytes, 0, &v.dev, &v.block);
        if (rc) return rc;
        std::memcpy(v.dims, dims, sizeof v.dims);
        v.dtype = dtype;
        if ((rc = take_event(&v.ready))) {
            put_block(v.dev, v.block);
            return rc;
        }
        hipError_t e;
        if (!pitch) {
            e = hipMemcpyAsync(v.dev, host, bytes, hipMemcpyHostToDevice, upload_);
        } else {
            hipMemcpy3DParms p{};
            p.srcPtr = make_hipPitchedPtr(const_cast<void*>(host), (size_t)pitch[0] * es,
                                          (size_t)dims[0], (size_t)(pitch[1] / pitch[0]));
            p.dstPtr = make_hipPitchedPtr(v.dev, (size_t)dims[0] * es, (size_t)dims[0],
                                          (size_t)dims[1]);
            p.extent = make_hipExtent((size_t)dims[0] * es, (size_t)dims[1], (size_t)dims[2]);
            p.kind = hipMemcpyHostToDevice;
            e = hipMemcpy3DAsync(&p, upload_);
        }
        if (e != hipSuccess || hipEventRecord(v.ready, upload_) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipStreamSynchronize(upload_);
            free_events_.push_back(v.ready);
            put_block(v.dev, v.block);
            return LNF_EHIP;
        }
        const uint64_t vid = next_vol_++;
        lru_.push_back(vid);
        v.lru = std::prev(lru_.end());
        vols_[vid] = v;
        ++uploads_;
        *id = vid;
        return LNF_OK;
    }

    int release(uint64_t id)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = vols_.find(id);
        if (it == vols_.end() || it->second.released) return LNF_ENOTFOUND;
        it->second.released = true;
        if (it->second.refs == 0) drop_volume(it);
        return LNF_OK;
    }

    int submit(uint64_t vid, int radius, void* host_out, int64_t arrival, uint64_t* ticket)
    {
        if (!ticket || radius < 1 || radius > LNF_RADIUS_MAX) return LNF_EINVAL;
        std::unique_lock<std::mutex> lk(mu_);
        if (stop_) return LNF_ECANCELED;
        auto it = vols_.find(vid);
        if (it == vols_.end() || it->second.released) return LNF_ENOTFOUND;
        Volume& v = it->second;
        // the volume and this request's output must fit under the cap together,
        // else the request could never be admitted
        const size_t vbytes = (size_t)v.dims[0] * v.dims[1] * v.dims[2] * (v.dtype == LNF_U8 ? 1 : 2);
        if (Arena::round(vbytes) + Arena::round(vbytes) > o_.cap_bytes) return LNF_EBUSY;
        v.refs += 1;
        touch(vid, v);
        Request r;
        r.vol = vid;
        r.radius = radius;
        r.host_out = host_out;
        r.arrival = arrival > 0 ? arrival : steady_ns();
        r.voxels = (uint64_t)v.dims[0] * v.dims[1] * v.dims[2];
        const uint64_t t = next_ticket_++;
        reqs_[t] = r;
        pending_.push_back(t);
        ++submitted_;
        if (first_arrival_ == 0 || r.arrival < first_arrival_) first_arrival_ = r.arrival;
        *ticket = t;
        lk.unlock();
        cv_.notify_all();
        return LNF_OK;
    }

    int poll(uint64_t t, int* done)
    {
        if (!done) return LNF_EINVAL;
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(t);
        if (it == reqs_.end()) return LNF_ENOTFOUND;
        *done = it->second.state == kDone;
        return *done ? it->second.status : LNF_OK;
    }

    int wait(uint64_t t, int timeout_ms)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto pred = [&] {
            auto it = reqs_.find(t);
            return it == reqs_.end() || it->second.state == kDone;
        };
        if (timeout_ms < 0) done_cv_.wait(lk, pred);
        else if (!done_cv_.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred))
            return LNF_ETIMEDOUT;
        auto it = reqs_.find(t);
        return it == reqs_.end() ? LNF_ENOTFOUND : it->second.status;
    }

    int cancel(uint64_t t)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(t);
        if (it == reqs_.end()) return LNF_ENOTFOUND;
        if (it->second.state != kPending) return LNF_EBUSY;
        pending_.erase(std::find(pending_.begin(), pending_.end(), t));
        finish(t, LNF_ECANCELED, 0);
        lk.unlock();
        done_cv_.notify_all();
        return LNF_OK;
    }

    int sync()
    {
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [&] { return pending_.empty() && flights_.empty(); });
        return LNF_OK;
    }

    int stats(lnf_server_stats_t* st, int reset)
    {
        if (!st) return LNF_EINVAL;
        std::unique_lock<std::mutex> lk(mu_);
        lnf_server_stats_t s{};
        s.submitted = submitted_;
        s.completed = completed_;
        s.failed = failed_;
        s.cancelled = cancelled_;
        s.batches = batches_;
        s.evictions = evictions_;
        s.uploads = uploads_;
        s.voxels = voxels_;
        s.bytes_in_use = arena_.reserved();
        s.peak_bytes = peak_;
        if (!lat_ms_.empty()) {
            std::vector<double> v = lat_ms_;
            auto pct = [&](double q) {
                const size_t k = std::min(v.size() - 1, (size_t)std::floor(q * (v.size() - 1) + 0.5));
                std::nth_element(v.begin(), v.begin() + k, v.end());
                return v[k];
            };
            s.p50_ms = pct(0.50);
            s.p99_ms = pct(0.99);
            s.max_ms = *std::max_element(v.begin(), v.end());
            double sum = 0;
            for (double x : v) sum += x;
            s.mean_ms = sum / v.size();
        }
        if (last_done_ > first_arrival_ && first_arrival_ > 0) {
            s.busy_s = (last_done_ - first_arrival_) * 1e-9;
            s.gvox_per_s = voxels_ / s.busy_s / 1e9;
        }
        *st = s;
        if (reset) {
            lat_ms_.clear();
            submitted_ = completed_ = failed_ = cancelled_ = batches_ = evictions_ = uploads_ = 0;
            voxels_ = 0;
            first_arrival_ = last_done_ = 0;
            peak_ = arena_.reserved();
        }
        return LNF_OK;
    }

private:
    // ---- memory -------------------------------------------------------------
    // A range of `bytes` for a volume or an output: free space first, then a
    // new chunk while the cap allows, then evicting idle volumes (never `keep`).
    int get_block(size_t bytes, uint64_t keep, void** p, size_t* block)
    {
        const size_t n = Arena::round(bytes);
        if (n > o_.cap_bytes) return LNF_EBUSY;
        for (;;) {
            if ((*p = arena_.take(n))) {
                *block = n;
                peak_ = std::max(peak_, arena_.reserved());
                return LNF_OK;
            }
            const int rc = arena_.grow(n, o_.cap_bytes);
            if (rc == LNF_OK) continue;
            if (rc == LNF_ENOMEM && arena_.reserved() == 0) return LNF_ENOMEM;
            if (!evict_one(keep)) return LNF_EBUSY;  // wait for requests to finish
        }
    }

    void put_block(void* p, size_t n) { arena_.give(p, n); }

    // Evict the least recently used idle volume: those whose upload has
    // finished first, then (waiting for the copy) those still being uploaded.
    bool evict_one(uint64_t keep)
    {
        for (int pass = 0; pass < 2; ++pass) {
            for (uint64_t id : lru_) {
                if (id == keep) continue;
                auto vit = vols_.find(id);
                if (vit->second.refs > 0) continue;
                if (pass == 0 && hipEventQuery(vit->second.ready) != hipSuccess) continue;
                drop_volume(vit);
                ++evictions_;
                return true;
            }
        }
        return false;
    }

    // Return a volume's range to the arena (after its upload has completed).
    void drop_volume(std::unordered_map<uint64_t, Volume>::iterator it)
    {
        Volume& v = it->second;
        (void)hipEventSynchronize(v.ready);
        free_events_.push_back(v.ready);
        put_block(v.dev, v.block);
        lru_.erase(v.lru);
        vols_.erase(it);
    }

    void touch(uint64_t id, Volume& v)
    {
        lru_.erase(v.lru);
        lru_.push_back(id);
        v.lru = std::prev(lru_.end());
    }

    int take_event(hipEvent_t* e)
    {
        if (!free_events_.empty()) {
            *e = free_events_.back();
            free_events_.pop_back();
            return LNF_OK;
        }
        return hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess ? LNF_OK : LNF_EHIP;
    }

    // ---- request life cycle --------------------------------------------------
    // End a request: release its output block and volume reference, record it.
    // `failure` counts an LNF_ECANCELED end as a failure (a failed batch) rather
    // than a cancellation.
    void finish(uint64_t t, int status, int64_t now, bool failure = false)
    {
        Request& r = reqs_[t];
        r.state = kDone;
        r.status = status;
        if (r.out) {
            put_block(r.out, r.block);
            r.out = nullptr;
        }
        auto vit = vols_.find(r.vol);
        if (vit != vols_.end()) {
            vit->second.refs -= 1;
            if (vit->second.refs == 0 && vit->second.released) drop_volume(vit);
        }
        if (status == LNF_OK) {
            ++completed_;
            voxels_ += r.voxels;
            lat_ms_.push_back((now - r.arrival) * 1e-6);
            last_done_ = std::max(last_done_, now);
        } else if (status == LNF_ECANCELED && !failure) {
            ++cancelled_;
        } else {
            ++failed_;
        }
    }

    // Whether another batch may go to the device now (the device queue bound).
    bool may_launch() const { return flights_.size() < 2 || inflight_vox_ < 2 * budget_; }

    // Admit pending requests in order while memory, max_batch and the voxel
    // budget allow; returns the admitted.
    std::vector<uint64_t> admit()
    {
        std::vector<uint64_t> got;
        const int cap = o_.mode == LNF_SERVE_FIFO ? 1 : o_.max_batch;
        uint64_t vox = 0;
        while (!pending_.empty() && (int)got.size() < cap) {
            const uint64_t t = pending_.front();
            Request& r = reqs_[t];
            if (!got.empty() && vox + r.voxels > budget_) break;  // starts the next batch
            const Volume& v = vols_[r.vol];
            const size_t bytes = (size_t)r.voxels * (v.dtype == LNF_U8 ? 1 : 2);
            if (get_block(bytes, r.vol, &r.out, &r.block) != LNF_OK) {
                // Nothing in flight or admitted in this pass will free memory
                // and every idle volume is already evicted: the request cannot
                // be admitted now, nor later.  End it so the queue moves on.
                if (!flights_.empty() || !got.empty()) break;  // wait for memory
                pending_.pop_front();
                finish(t, LNF_EBUSY, steady_ns(), true);
                done_cv_.notify_all();
                continue;
            }
            r.state = kInFlight;
            pending_.pop_front();
            got.push_back(t);
            vox += r.voxels;
        }
        return got;
    }

    void launch(std::vector<uint64_t>& ts)
    {
        hipStream_t s = streams_[next_stream_];
        next_stream_ = (next_stream_ + 1) % (int)streams_.size();
        ++batches_;
        std::vector<lnf_job> jobs;
        std::vector<uint64_t> seen;
        for (uint64_t t : ts) {
            Request& r = reqs_[t];
            Volume& v = vols_[r.vol];
            if (std::find(seen.begin(), seen.end(), r.vol) == seen.end()) {
                (void)hipStreamWaitEvent(s, v.ready, 0);
                seen.push_back(r.vol);
            }
            lnf_job j;
            j.in = v.dev;
            j.out = r.out;
            std::memcpy(j.dims, v.dims, sizeof j.dims);
            j.dtype = v.dtype;
            j.radius = r.radius;
            jobs.push_back(j);
        }
        int rc = LNF_OK;
        if (o_.fail_batch > 0 && batches_ == (uint64_t)o_.fail_batch) rc = LNF_ECANCELED;
        if (rc == LNF_OK) {
            // a micro-batch of one is a plain launch: no table upload
            if (o_.mode == LNF_SERVE_FIFO || jobs.size() == 1)
                rc = lnf_filter(h_, jobs[0].in, jobs[0].dims, jobs[0].dtype, jobs[0].radius,
                                jobs[0].out, s);
            else
                rc = lnf_filter_batch(h_, jobs.data(), (int)jobs.size(), s);
        }
        for (size_t i = 0; rc == LNF_OK && i < ts.size(); ++i) {
            Request& r = reqs_[ts[i]];
            if (r.host_out) {
                const size_t bytes = (size_t)r.voxels * (jobs[i].dtype == LNF_U8 ? 1 : 2);
                if (hipMemcpyAsync(r.host_out, r.out, bytes, hipMemcpyDeviceToHost, s) != hipSuccess)
                    rc = LNF_EHIP;
            }
        }
        Flight f;
        f.tickets = ts;
        for (uint64_t t : ts) f.voxels += reqs_[t].voxels;
        if (rc == LNF_OK) rc = take_event(&f.done);
        if (rc == LNF_OK && hipEventRecord(f.done, s) != hipSuccess) rc = LNF_EHIP;
        if (rc != LNF_OK) {
            (void)hipGetLastError();
            (void)hipStreamSynchronize(s);  // nothing of this batch may still touch its blocks
            if (f.done) free_events_.push_back(f.done);
            const int64_t now = steady_ns();
            for (uint64_t t : ts) finish(t, rc, now, true);
            done_cv_.notify_all();
            return;
        }
        inflight_vox_ += f.voxels;
        flights_.push_back(std::move(f));
    }

    bool reap()
    {
        bool any = false;
        for (auto it = flights_.begin(); it != flights_.end();) {
            const hipError_t q = hipEventQuery(it->done);
            if (q == hipErrorNotReady) {
                ++it;
                continue;
            }
            const int64_t now = steady_ns();
            const int status = q == hipSuccess ? LNF_OK : LNF_EHIP;
            if (q != hipSuccess) (void)hipGetLastError();
            for (uint64_t t : it->tickets) finish(t, status, now);
            free_events_.push_back(it->done);
            inflight_vox_ -= it->voxels;
            it = flights_.erase(it);
            any = true;
        }
        if (any) done_cv_.notify_all();
        return any;
    }

    void loop()
    {
        DeviceGuard dg(h_->device);
        std::unique_lock<std::mutex> lk(mu_);
        while (true) {
            bool progress = reap();
            if (!pending_.empty() && may_launch()) {
                std::vector<uint64_t> ts = admit();
                if (!ts.empty()) {
                    launch(ts);
                    progress = true;
                }
            }
            if (stop_ && pending_.empty() && flights_.empty()) break;
            if (!progress) {
                if (flights_.empty() && pending_.empty())
                    cv_.wait(lk, [&] { return stop_ || !pending_.empty(); });
                else
                    cv_.wait_for(lk, std::chrono::microseconds(20));
            }
        }
        done_cv_.notify_all();
    }

    lnf_handle h_;
    lnf_server_options o_;
    uint64_t budget_;            // voxel budget of one micro-batch
    uint64_t inflight_vox_ = 0;  // voxels of the batches in flight
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::thread worker_;
    bool stop_ = false;
    std::vector<hipStream_t> streams_;
    hipStream_t upload_ = nullptr;
    int next_stream_ = 0;

    std::unordered_map<uint64_t, Volume> vols_;
    std::list<uint64_t> lru_;
    std::unordered_map<uint64_t, Request> reqs_;
    std::deque<uint64_t> pending_;
    std::list<Flight> flights_;
    Arena arena_;
    std::vector<hipEvent_t> free_events_;
    size_t peak_ = 0;  // largest device footprint (arena chunks) seen
    uint64_t next_vol_ = 1, next_ticket_ = 1;

    uint64_t submitted_ = 0, completed_ = 0, failed_ = 0, cancelled_ = 0, batches_ = 0;
    uint64_t evictions_ = 0, uploads_ = 0, voxels_ = 0;
    int64_t first_arrival_ = 0, last_done_ = 0;
    std::vector<double> lat_ms_;
};

}  // namespace lnf

struct lnf_server {
    lnf::Server* impl;
};

using namespace lnf;

extern "C" {

int64_t lnf_server_now_ns(void) { return steady_ns(); }

int lnf_server_create(lnf_handle h, const lnf_server_options* opt, lnf_server_handle* srv)
{
    if (!h || !srv) return LNF_EINVAL;
    *srv = nullptr;
    lnf_server_options o{sizeof(lnf_server_options), LNF_SERVE_BATCHED, 200ull << 30, 4, 256, 0, 0};
    if (opt) {
        if (opt->size < sizeof(lnf_server_options)) return LNF_EINVAL;
        o = *opt;
    }
    if ((o.mode != LNF_SERVE_BATCHED && o.mode != LNF_SERVE_FIFO) || o.cap_bytes == 0 ||
        o.n_streams < 1 || o.n_streams > 16 || o.max_batch < 1 || o.max_batch > LNF_BATCH_MAX ||
        o.fail_batch < 0 || o.batch_mvox < 0 || o.batch_mvox > (1 << 20))
        return LNF_EINVAL;
    Server* s = new (std::nothrow) Server(h, o);
    if (!s) return LNF_ENOMEM;
    const int rc = s->init();
    if (rc) {
        delete s;
        return rc;
    }
    lnf_server* w = new (std::nothrow) lnf_server{s};
    if (!w) {
        delete s;
        return LNF_ENOMEM;
    }
    *srv = w;
    return LNF_OK;
}

int lnf_server_destroy(lnf_server_handle srv)
{
    if (!srv) return LNF_OK;
    delete srv->impl;
    delete srv;
    return LNF_OK;
}

int lnf_server_put_volume(lnf_server_handle srv, const void* host, const int64_t dims[3], int dtype,
                          const int64_t* host_pitch, uint64_t* vol_id)
{
    if (!srv) return LNF_EINVAL;
    return srv->impl->put(host, dims, dtype, host_pitch, vol_id);
}

int lnf_server_release(lnf_server_handle srv, uint64_t vol_id)
{
    if (!srv) return LNF_EINVAL;
    return srv->impl->release(vol_id);
}

int lnf_server_submit(lnf_server_handle srv, uint64_t vol_id, int radius, void* host_out,
                      int64_t arrival_ns, uint64_t* ticket)
{
    if (!srv) return LNF_EINVAL;
    return srv->impl->submit(vol_id, radius, host_out, arrival_ns, ticket);
}

int lnf_server_poll(lnf_server_handle srv, uint64_t ticket, int* done)
{
    if (!srv) return LNF_EINVAL;
    return srv->impl->poll(ticket, done);
}

int lnf_server_wait(lnf_server_handle srv, uint64_t ticket, int timeout_ms)
{
    if (!srv) return LNF_EINVAL;
    return srv->impl->wait(ticket, timeout_ms);
}

int lnf_server_cancel(lnf_server_handle srv, uint64_t ticket)
{
    if (!srv) return LNF_EINVAL;
    return srv->impl->cancel(ticket);
}

int lnf_server_sync(lnf_server_handle srv)
{
    if (!srv) return LNF_EINVAL;
    return srv->impl->sync();
}

int lnf_server_stats(lnf_server_handle srv, lnf_server_stats_t* st, int reset)
{
    if (!srv) return LNF_EINVAL;
    return srv->impl->stats(st, reset);
}

}  // extern "C"
