// Sort server: admission of sort requests by an HBM budget, continuous
// batching of short requests into batched segmented sorts, and overlapping
// jobs on several HIP streams (the request loop declared in evosort.h).
//
// One scheduler thread owns the device work.  Client threads submit, poll,
// wait, copy out and release; everything shared is guarded by one mutex.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "capi_internal.hpp"
#include "evosort.h"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int key_bytes_of(int dtype)
{
    switch (dtype) {
    case EVOSORT_INT32:
    case EVOSORT_UINT32:
    case EVOSORT_FLOAT32:
        return 4;
    case EVOSORT_INT64:
    case EVOSORT_FLOAT64:
        return 8;
    default:
        return 0;
    }
}

// First-fit allocator over byte offsets [0, size) of the arena; free ranges
// are kept sorted by offset and merged with their neighbours on release.
class Arena {
public:
    void reset(size_t size)
    {
        free_.clear();
        if (size)
            free_[0] = size;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes)
                continue;
            *off = it->first;
            const size_t rest = it->second - bytes, next = it->first + bytes;
            free_.erase(it);
            if (rest)
                free_[next] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes ? bytes : 1);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
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
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

struct Range {
    size_t off = 0, bytes = 0;
};

// One gathered request of a batch: copy `bytes` from src to the batch
// buffer at byte offset dst_off.
struct GatherItem {
    const void* src;
    uint64_t dst_off;
    uint64_t bytes;
};

// One workgroup per request; every key is 4 or 8 bytes and every pointer
// and offset is a multiple of 4, so 4-byte words are copied, eight in flight
// per thread (all loads issued before the first store).
__global__ __launch_bounds__(256) void gather_kernel(const GatherItem* __restrict__ items,
                                                     unsigned char* __restrict__ dst)
{
    const GatherItem it = items[blockIdx.x];
    const uint32_t* s = reinterpret_cast<const uint32_t*>(it.src);
    uint32_t* d = reinterpret_cast<uint32_t*>(dst + it.dst_off);
    const uint64_t words = it.bytes / 4;
    const uint64_t bd = blockDim.x;
    uint64_t i = threadIdx.x;
    for (; i + 7 * bd < words; i += 8 * bd) {
        const uint32_t w0 = s[i], w1 = s[i + bd], w2 = s[i + 2 * bd], w3 = s[i + 3 * bd];
        const uint32_t w4 = s[i + 4 * bd], w5 = s[i + 5 * bd], w6 = s[i + 6 * bd], w7 = s[i + 7 * bd];
        __builtin_amdgcn_sched_barrier(0);
        d[i] = w0;
        d[i + bd] = w1;
        d[i + 2 * bd] = w2;
        d[i + 3 * bd] = w3;
        d[i + 4 * bd] = w4;
        d[i + 5 * bd] = w5;
        d[i + 6 * bd] = w6;
        d[i + 7 * bd] = w7;
    }
    for (; i < words; i += bd)
        d[i] = s[i];
}

struct Request {
    int dtype = 0;
    const void* in = nullptr;
    int64_t n = 0;
    double t_submit = 0, t_admit = -1, t_done = -1;
    int status = EVOSORT_ERR_PENDING;
    void* out = nullptr;  // result (in the arena) once done
    int64_t job = -1;
};

struct Job {
    std::vector<uint64_t> reqs;
    Range result;    // freed when every request of the job is released
    Range scratch;   // freed when the job finishes
    int slot = -1;
    int status = EVOSORT_OK;
    int unreleased = 0;
    std::vector<hipEvent_t> readers;  // copies out of `result` queued on client streams (copy_out)
};

// Arena ranges of released jobs whose result is still being copied out on a
// client stream: freed once every one of those copies has finished.
struct Deferred {
    Range result;
    std::vector<hipEvent_t> readers;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int64_t job = -1;           // running job, or -1
    unsigned char* staging = nullptr;  // pinned host: descriptors and offsets of a batch
    size_t desc_off = 0;        // arena offset of the device copy of the staging area
    uint32_t* err_host = nullptr;  // pinned, device-mapped word the slot's kernels set on a device error
    uint32_t* err_dev = nullptr;   // the same word as kernels address it
};

}  // namespace

struct evosort_server {
    evosort_server_config cfg{};
    evosort_params batch_params{};
    int device = 0;
    unsigned char* arena_base = nullptr;
    size_t usable = 0;  // arena bytes available to requests (after the slots' descriptor areas)
    Arena arena;
    std::vector<Slot> slots;
    size_t staging_bytes = 0;

    std::mutex mu;
    std::condition_variable cv_work;  // submissions, releases, stop
    std::condition_variable cv_done;  // finished requests
    std::thread worker;
    bool stop = false;

    uint64_t next_id = 1;
    int64_t next_job = 0;
    std::deque<uint64_t> waiting;
    std::unordered_map<uint64_t, Request> reqs;
    std::unordered_map<int64_t, Job> jobs;
    std::vector<Deferred> deferred;
    std::vector<hipEvent_t> event_pool;
    evosort_server_stats st{};
    uint32_t running = 0;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now_ms() const
    {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    void note_bytes()
    {
        st.bytes_in_use = arena.used();
        if (st.bytes_in_use > st.peak_bytes)
            st.peak_bytes = st.bytes_in_use;
    }

    // Footprint of a request run alone: output plus evosort_sort scratch.
    bool single_footprint(int dtype, int64_t n, size_t* out_bytes, size_t* temp_bytes) const
    {
        size_t tb = 0;
        if (evosort_temp_bytes(EVOSORT_OP_SORT, dtype, n, 0, &cfg.params, &tb) != EVOSORT_OK)
            return false;
        *out_bytes = (size_t)n * (size_t)key_bytes_of(dtype);
        *temp_bytes = tb;
        return true;
    }

    void finish_job(int64_t jid, int status)
    {
        Job& j = jobs[jid];
        const double t = now_ms();
        j.status = status;
        for (uint64_t r : j.reqs) {
            Request& q = reqs[r];
            q.status = status;
            q.t_done = t;
            if (status == EVOSORT_OK) {
                st.completed++;
                st.keys_completed += (uint64_t)q.n;
            } else {
                st.failed++;
            }
        }
        if (j.scratch.bytes) {
            arena.release(j.scratch.off, j.scratch.bytes);
            j.scratch = Range{};
        }
        if (j.slot >= 0) {
            slots[j.slot].job = -1;
            running--;
        }
        note_bytes();
        cv_done.notify_all();
    }

    hipEvent_t get_event()
    {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return e;
    }

    // Frees a released job's result now, or once the copies out of it that
    // clients queued have finished.
    void free_result(Job& j)
    {
        if (!j.result.bytes)
            return;
        if (j.readers.empty()) {
            arena.release(j.result.off, j.result.bytes);
        } else {
            deferred.push_back(Deferred{j.result, std::move(j.readers)});
            j.readers.clear();
        }
        j.result = Range{};
    }

    // Frees the deferred ranges whose copies have all finished (wait: block
    // until they have).
    void reap_deferred(bool wait)
    {
        for (size_t i = 0; i < deferred.size();) {
            Deferred& d = deferred[i];
            bool done = true;
            for (hipEvent_t e : d.readers) {
                const hipError_t q = wait ? hipEventSynchronize(e) : hipEventQuery(e);
                if (q == hipErrorNotReady) {
                    done = false;
                    break;
                }
                (void)hipGetLastError();  // a failed copy frees its range all the same
            }
            if (!done) {
                ++i;
                continue;
            }
            for (hipEvent_t e : d.readers)
                event_pool.push_back(e);
            arena.release(d.result.off, d.result.bytes);
            deferred[i] = std::move(deferred.back());
            deferred.pop_back();
        }
        note_bytes();
    }

    // Arena offsets count from the end of the slots' descriptor areas.
    void* ptr(const Range& r) const { return arena_base + (size_t)cfg.streams * staging_bytes + r.off; }

    // Admit the request at the head of the queue (and, for a short one, the
    // short requests of the same key type among the waiting ones) on slot s.
    // Returns false when the head does not fit in the arena yet.
    bool admit(int s)
    {
        const uint64_t head = waiting.front();
        Request& h = reqs[head];
        const int kb = key_bytes_of(h.dtype);
        const bool batchable = cfg.batch_max_keys > 0 && (uint64_t)h.n <= cfg.batch_max_keys;
        Slot& sl = slots[s];
        Job job;
        job.slot = s;
        if (!batchable) {
            size_t ob = 0, tb = 0;
            if (!single_footprint(h.dtype, h.n, &ob, &tb))
                return false;
            Range ro, rt;
            if (!arena.alloc(ob, &ro.off))
                return false;
            ro.bytes = ob;
            if (!arena.alloc(tb, &rt.off)) {
                arena.release(ro.off, ro.bytes);
                return false;
            }
            rt.bytes = tb;
            waiting.pop_front();
            job.reqs.push_back(head);
            job.result = ro;
            job.scratch = rt;
            const int64_t jid = next_job++;
            jobs[jid] = job;
            h.job = jid;
            h.out = ptr(ro);
            h.t_admit = now_ms();
            sl.job = jid;
            running++;
            st.jobs++;
            if (running > st.max_concurrent_jobs)
                st.max_concurrent_jobs = running;
            note_bytes();
            __atomic_store_n(sl.err_host, 0u, __ATOMIC_RELEASE);  // the slot is idle: no kernel writes it now
            int rc = evosort::server_sort(h.dtype, h.in, h.out, h.n, ptr(rt), rt.bytes, &cfg.params, sl.stream,
                                          sl.err_dev);
            if (rc == EVOSORT_OK && hipEventRecord(sl.done, sl.stream) != hipSuccess)
                rc = EVOSORT_ERR_HIP;
            if (rc != EVOSORT_OK)
                finish_job(jid, rc);
            return true;
        }
        // a batch: the head plus same-type short requests, in arrival order
        std::vector<uint64_t> pick;
        uint64_t total = 0;
        const size_t max_req = cfg.batch_max_requests;
        for (auto it = waiting.begin(); it != waiting.end() && pick.size() < max_req; ++it) {
            const Request& q = reqs[*it];
            if (q.dtype != h.dtype || (uint64_t)q.n > cfg.batch_max_keys)
                continue;
            pick.push_back(*it);
            total += (uint64_t)q.n;
        }
        // the batch's buffer and scratch; a batch that does not fit is cut
        // to its first half (arrival order) until it fits or the head alone
        // does not
        Range rb, rt;
        for (;;) {
            total = 0;
            for (uint64_t r : pick)
                total += (uint64_t)reqs[r].n;
            size_t tb = 0;
            if (evosort_segmented_temp_bytes(h.dtype, (int64_t)total, (int64_t)pick.size(), 0, &batch_params,
                                             &tb) != EVOSORT_OK)
                return false;
            rb.bytes = (size_t)total * (size_t)kb;
            rt.bytes = tb;
            if (arena.alloc(rb.bytes, &rb.off)) {
                if (arena.alloc(rt.bytes, &rt.off))
                    break;
                arena.release(rb.off, rb.bytes);
            }
            if (pick.size() == 1)
                return false;
            pick.resize(pick.size() / 2);
        }
        const int64_t nseg = (int64_t)pick.size();
        // staging: GatherItem[nseg], then int64 offsets[nseg + 1]
        GatherItem* items = reinterpret_cast<GatherItem*>(sl.staging);
        int64_t* offs = reinterpret_cast<int64_t*>(sl.staging + (size_t)nseg * sizeof(GatherItem));
        unsigned char* buf = reinterpret_cast<unsigned char*>(ptr(rb));
        const double t = now_ms();
        const int64_t jid = next_job++;
        uint64_t pos = 0;
        for (int64_t i = 0; i < nseg; ++i) {
            Request& q = reqs[pick[(size_t)i]];
            items[i] = GatherItem{q.in, pos * (uint64_t)kb, (uint64_t)q.n * (uint64_t)kb};
            offs[i] = (int64_t)pos;
            q.out = buf + pos * (uint64_t)kb;
            q.job = jid;
            q.t_admit = t;
            pos += (uint64_t)q.n;
        }
        offs[nseg] = (int64_t)pos;
        // remove the picked requests from the queue (they are in queue order)
        {
            size_t k = 0;
            std::deque<uint64_t> rest;
            for (uint64_t r : waiting) {
                if (k < pick.size() && r == pick[k])
                    ++k;
                else
                    rest.push_back(r);
            }
            waiting.swap(rest);
        }
        job.reqs = pick;
        job.result = rb;
        job.scratch = rt;
        jobs[jid] = job;
        sl.job = jid;
        running++;
        st.jobs++;
        st.batched_requests += (uint64_t)nseg;
        if (running > st.max_concurrent_jobs)
            st.max_concurrent_jobs = running;
        note_bytes();

        unsigned char* desc = arena_base + sl.desc_off;
        const size_t desc_bytes = (size_t)nseg * sizeof(GatherItem) + (size_t)(nseg + 1) * sizeof(int64_t);
        int rc = EVOSORT_OK;
        __atomic_store_n(sl.err_host, 0u, __ATOMIC_RELEASE);
        if (hipMemcpyAsync(desc, sl.staging, desc_bytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
            rc = EVOSORT_ERR_HIP;
        if (rc == EVOSORT_OK && total > 0) {
            (void)hipGetLastError();
            hipLaunchKernelGGL(gather_kernel, dim3((uint32_t)nseg), dim3(256), 0, sl.stream,
                               reinterpret_cast<const GatherItem*>(desc), buf);
            if (hipGetLastError() != hipSuccess)
                rc = EVOSORT_ERR_HIP;
        }
        if (rc == EVOSORT_OK)
            rc = evosort::server_segmented_sort(
                h.dtype, buf, buf, (int64_t)total,
                reinterpret_cast<const int64_t*>(desc + (size_t)nseg * sizeof(GatherItem)), nseg, ptr(rt), rt.bytes,
                &batch_params, sl.stream, sl.err_dev);
        if (rc == EVOSORT_OK && hipEventRecord(sl.done, sl.stream) != hipSuccess)
            rc = EVOSORT_ERR_HIP;
        if (rc != EVOSORT_OK)
            finish_job(jid, rc);
        return true;
    }

    void loop()
    {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            // retire finished jobs
            for (size_t s = 0; s < slots.size(); ++s) {
                if (slots[s].job < 0)
                    continue;
                const hipError_t q = hipEventQuery(slots[s].done);
                if (q == hipSuccess) {
                    // a device-side failure (a look-back wait out of spins) fails the job
                    const uint32_t bits = __atomic_load_n(slots[s].err_host, __ATOMIC_ACQUIRE);
                    finish_job(slots[s].job, evosort::status_of_error_bits(bits));
                } else if (q != hipErrorNotReady) {
                    finish_job(slots[s].job, EVOSORT_ERR_HIP);
                }
            }
            if (!deferred.empty())
                reap_deferred(false);
            // admit in arrival order while a slot is free and the head fits
            if (!stop) {
                for (size_t s = 0; s < slots.size() && !waiting.empty(); ++s) {
                    if (slots[s].job >= 0)
                        continue;
                    if (!admit((int)s))
                        break;
                }
            }
            st.waiting = (uint32_t)waiting.size();
            if (stop && running == 0)
                break;
            if (running > 0 || !deferred.empty()) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(5));
                lk.lock();
            } else {
                cv_work.wait_for(lk, std::chrono::milliseconds(1));
            }
        }
        // requests never admitted are dropped
        for (uint64_t r : waiting) {
            reqs[r].status = EVOSORT_ERR_INVALID_ARG;
            reqs[r].t_done = now_ms();
        }
        waiting.clear();
        cv_done.notify_all();
    }
};

extern "C" {

void evosort_server_default_config(evosort_server_config* cfg)
{
    if (!cfg)
        return;
    memset(cfg, 0, sizeof(*cfg));
    cfg->struct_size = sizeof(*cfg);
    cfg->streams = 4;
    cfg->hbm_budget_bytes = (uint64_t)1 << 30;
    cfg->batch_max_keys = 65536;
    cfg->batch_max_requests = 2048;
    evosort_default_params(&cfg->params);
}

evosort_status evosort_server_create(const evosort_server_config* cfg, evosort_server** out)
{
    if (!cfg || !out || cfg->struct_size != sizeof(evosort_server_config))
        return EVOSORT_ERR_INVALID_ARG;
    *out = nullptr;
    if (cfg->streams < 1 || cfg->streams > 16 || cfg->batch_max_requests < 1 || cfg->batch_max_requests > 8192 ||
        cfg->batch_max_keys >= ((uint64_t)1 << 30))
        return EVOSORT_ERR_INVALID_ARG;
    size_t probe = 0;
    if (evosort_temp_bytes(EVOSORT_OP_SORT, EVOSORT_INT32, 1, 0, &cfg->params, &probe) != EVOSORT_OK)
        return EVOSORT_ERR_INVALID_ARG;
    auto* S = new evosort_server();
    S->cfg = *cfg;
    evosort_default_params(&S->batch_params);
    S->batch_params.fallback_threshold = cfg->params.fallback_threshold;
    S->batch_params.descending = cfg->params.descending;
    S->staging_bytes =
        align_up((size_t)cfg->batch_max_requests * sizeof(GatherItem) + ((size_t)cfg->batch_max_requests + 1) * 8);
    const size_t reserved = (size_t)cfg->streams * S->staging_bytes;
    if (cfg->hbm_budget_bytes <= reserved + kAlign) {
        delete S;
        return EVOSORT_ERR_INVALID_ARG;
    }
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return EVOSORT_ERR_HIP;
    }
    void* base = nullptr;
    if (hipMalloc(&base, (size_t)cfg->hbm_budget_bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete S;
        return EVOSORT_ERR_HIP;
    }
    S->arena_base = reinterpret_cast<unsigned char*>(base);
    S->usable = (size_t)cfg->hbm_budget_bytes - reserved;
    S->arena.reset(S->usable & ~(kAlign - 1));
    S->st.budget_bytes = cfg->hbm_budget_bytes;
    S->slots.resize(cfg->streams);
    bool ok = true;
    for (uint32_t i = 0; i < cfg->streams && ok; ++i) {
        Slot& sl = S->slots[i];
        sl.desc_off = (size_t)i * S->staging_bytes;
        ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&sl.staging), S->staging_bytes, hipHostMallocDefault) ==
                 hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&sl.err_host), 64, hipHostMallocMapped | hipHostMallocCoherent) ==
                 hipSuccess &&
             hipHostGetDevicePointer(reinterpret_cast<void**>(&sl.err_dev), sl.err_host, 0) == hipSuccess;
        if (sl.err_host)
            *sl.err_host = 0;
    }
    if (!ok) {
        (void)hipGetLastError();
        for (Slot& sl : S->slots) {
            if (sl.stream)
                (void)hipStreamDestroy(sl.stream);
            if (sl.done)
                (void)hipEventDestroy(sl.done);
            if (sl.staging)
                (void)hipHostFree(sl.staging);
            if (sl.err_host)
                (void)hipHostFree(sl.err_host);
        }
        (void)hipFree(base);
        delete S;
        return EVOSORT_ERR_HIP;
    }
    S->worker = std::thread([S] { S->loop(); });
    *out = S;
    return EVOSORT_OK;
}

evosort_status evosort_server_destroy(evosort_server* S)
{
    if (!S)
        return EVOSORT_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    S->worker.join();
    for (Slot& sl : S->slots) {
        (void)hipStreamSynchronize(sl.stream);
        (void)hipStreamDestroy(sl.stream);
        (void)hipEventDestroy(sl.done);
        (void)hipHostFree(sl.staging);
        (void)hipHostFree(sl.err_host);
    }
    // copies out of the arena that clients queued must end before it is freed
    S->reap_deferred(true);
    for (auto& kv : S->jobs)
        for (hipEvent_t e : kv.second.readers) {
            (void)hipEventSynchronize(e);
            S->event_pool.push_back(e);
        }
    for (hipEvent_t e : S->event_pool)
        (void)hipEventDestroy(e);
    (void)hipFree(S->arena_base);
    delete S;
    return EVOSORT_OK;
}

evosort_status evosort_server_submit(evosort_server* S, int dtype, const void* keys_in, int64_t n, uint64_t* id)
{
    if (!S || !id || n < 0 || (n > 0 && !keys_in))
        return EVOSORT_ERR_INVALID_ARG;
    const int kb = key_bytes_of(dtype);
    if (!kb)
        return EVOSORT_ERR_UNSUPPORTED_DTYPE;
    // could it ever fit?  (alone: output + scratch, or as a batch of one)
    size_t ob = 0, tb = 0;
    if (!S->single_footprint(dtype, n, &ob, &tb))
        return EVOSORT_ERR_INVALID_ARG;
    size_t need = align_up(ob ? ob : 1) + align_up(tb ? tb : 1);
    if (S->cfg.batch_max_keys > 0 && (uint64_t)n <= S->cfg.batch_max_keys) {
        size_t sb = 0;
        if (evosort_segmented_temp_bytes(dtype, n, 1, 0, &S->batch_params, &sb) != EVOSORT_OK)
            return EVOSORT_ERR_INVALID_ARG;
        need = align_up(ob ? ob : 1) + align_up(sb ? sb : 1);
    }
    if (need > S->usable)
        return EVOSORT_ERR_OVER_BUDGET;
    std::lock_guard<std::mutex> g(S->mu);
    const uint64_t rid = S->next_id++;
    Request q;
    q.dtype = dtype;
    q.in = keys_in;
    q.n = n;
    q.t_submit = S->now_ms();
    S->st.submitted++;
    if (n == 0) {  // nothing to sort
        q.status = EVOSORT_OK;
        q.t_admit = q.t_done = q.t_submit;
        S->st.completed++;
        S->reqs[rid] = q;
    } else {
        S->reqs[rid] = q;
        S->waiting.push_back(rid);
        S->st.waiting = (uint32_t)S->waiting.size();
    }
    *id = rid;
    S->cv_work.notify_all();
    return EVOSORT_OK;
}

evosort_status evosort_server_result(evosort_server* S, uint64_t id, const void** keys_out)
{
    if (!S)
        return EVOSORT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end())
        return EVOSORT_ERR_INVALID_ARG;
    if (it->second.status == EVOSORT_OK && keys_out)
        *keys_out = it->second.out;
    return (evosort_status)it->second.status;
}

evosort_status evosort_server_wait(evosort_server* S, uint64_t id, const void** keys_out)
{
    if (!S)
        return EVOSORT_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end())
        return EVOSORT_ERR_INVALID_ARG;
    S->cv_done.wait(lk, [&] { return S->reqs[id].status != EVOSORT_ERR_PENDING; });
    const Request& q = S->reqs[id];
    if (q.status == EVOSORT_OK && keys_out)
        *keys_out = q.out;
    return (evosort_status)q.status;
}

evosort_status evosort_server_copy_out(evosort_server* S, uint64_t id, void* dst, void* stream)
{
    if (!S)
        return EVOSORT_ERR_INVALID_ARG;
    // The copy is queued on the client's stream; an event recorded after it
    // keeps the request's arena range from being reused (after a release)
    // until the copy has run.
    hipStream_t cs = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end())
        return EVOSORT_ERR_INVALID_ARG;
    const Request& q = it->second;
    if (q.status != EVOSORT_OK)
        return (evosort_status)q.status;
    if (q.n == 0)
        return EVOSORT_OK;
    if (!dst)
        return EVOSORT_ERR_INVALID_ARG;
    auto jt = S->jobs.find(q.job);
    if (jt == S->jobs.end())
        return EVOSORT_ERR_INVALID_ARG;
    hipEvent_t e = S->get_event();
    if (!e)
        return EVOSORT_ERR_HIP;
    if (hipMemcpyAsync(dst, q.out, (size_t)q.n * key_bytes_of(q.dtype), hipMemcpyDeviceToDevice, cs) != hipSuccess ||
        hipEventRecord(e, cs) != hipSuccess) {
        (void)hipGetLastError();
        // the copy may be queued; wait for the stream rather than lose track of it
        (void)hipStreamSynchronize(cs);
        S->event_pool.push_back(e);
        return EVOSORT_ERR_HIP;
    }
    jt->second.readers.push_back(e);
    return EVOSORT_OK;
}

evosort_status evosort_server_times(evosort_server* S, uint64_t id, double* submit_ms, double* admit_ms,
                                    double* done_ms)
{
    if (!S)
        return EVOSORT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end())
        return EVOSORT_ERR_INVALID_ARG;
    if (submit_ms)
        *submit_ms = it->second.t_submit;
    if (admit_ms)
        *admit_ms = it->second.t_admit;
    if (done_ms)
        *done_ms = it->second.t_done;
    return it->second.status == EVOSORT_ERR_PENDING ? EVOSORT_ERR_PENDING : EVOSORT_OK;
}

evosort_status evosort_server_release(evosort_server* S, uint64_t id)
{
    if (!S)
        return EVOSORT_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> g(S->mu);
        auto it = S->reqs.find(id);
        if (it == S->reqs.end())
            return EVOSORT_ERR_INVALID_ARG;
        if (it->second.status == EVOSORT_ERR_PENDING)
            return EVOSORT_ERR_PENDING;
        const int64_t jid = it->second.job;
        S->reqs.erase(it);
        S->st.released++;
        if (jid >= 0) {
            auto jt = S->jobs.find(jid);
            if (jt != S->jobs.end()) {
                Job& j = jt->second;
                j.unreleased = 0;
                for (uint64_t r : j.reqs)
                    j.unreleased += S->reqs.count(r) ? 1 : 0;
                if (j.unreleased == 0) {
                    S->free_result(j);
                    if (j.scratch.bytes)
                        S->arena.release(j.scratch.off, j.scratch.bytes);
                    S->jobs.erase(jt);
                    S->reap_deferred(false);  // copies that already ran free their ranges now
                }
            }
        }
    }
    S->cv_work.notify_all();
    return EVOSORT_OK;
}

evosort_status evosort_server_drain(evosort_server* S)
{
    if (!S)
        return EVOSORT_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] {
        if (!S->waiting.empty() || S->running > 0)
            return false;
        for (auto& kv : S->reqs)
            if (kv.second.status == EVOSORT_ERR_PENDING)
                return false;
        return true;
    });
    return EVOSORT_OK;
}

evosort_status evosort_server_get_stats(evosort_server* S, evosort_server_stats* out)
{
    if (!S || !out)
        return EVOSORT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(S->mu);
    S->reap_deferred(false);
    *out = S->st;
    out->bytes_in_use = S->arena.used();
    out->waiting = (uint32_t)S->waiting.size();
    return EVOSORT_OK;
}

}  // extern "C"
