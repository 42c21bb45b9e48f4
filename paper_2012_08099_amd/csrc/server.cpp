// Served loop: admission by device-memory budget, continuous batching of small
// requests, several streams in flight, completion with timestamps.  Every request is
// the same exact computation as dpm_moments (eq. 2 via the projections of Section 3.1
// and the recombination of Section 3.2); this file only schedules them.
//
// One worker thread owns all device work.  submit() appends to an incoming queue;
// the worker moves requests to a FIFO pending list, admits them when their arena
// blocks fit, launches them (batched or single) on the stream with the fewest jobs in
// flight, and retires jobs whose completion event has fired: results are copied from
// pinned staging into the caller's buffers, arena blocks are released, and a
// completion is queued for poll().
//
// Residency: a request submitted with keep_resident keeps, after completion, the 2D
// moments of each side of each of its projection images (collapsed from the power-sum
// tiles by a small kernel on the job's stream) in an arena block.  Such entries are
// evicted least recently used first when a job cannot be admitted otherwise; a query
// recombines an entry (Section 3.2) for any order up to the request's without reading
// the volume again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/dpm.h"
#include "dpm_common.h"
#include "kernels.h"
#include "resident.h"

namespace dpm {
int batched_run(const void *packed, const dpm_roi *rois, int n_rois, int max_order, const dpm_out *out_device,
                void *workspace, size_t ws_bytes, void *stream, bool allow_graphs);  // batched.cpp
int batched_partials(const dpm_roi *rois, int n_rois, int max_order, int i, size_t *part_off, size_t *rd_off,
                     int *nlr);  // batched.cpp
int single_partials(const int64_t dims[3], dpm_dtype dtype, int max_order, size_t *part_off,
                    int32_t tile0[NSLOT + 1], int *nlr);  // dpm_api.cpp
int batched_ensure_tables();  // dpm_api.cpp
}  // namespace dpm

namespace {

double now_ms_impl() {
    using namespace std::chrono;
    static const steady_clock::time_point t0 = steady_clock::now();
    return duration<double, std::milli>(steady_clock::now() - t0).count();
}

constexpr size_t kAlign = 256;
size_t al(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing on release.
class Arena {
public:
    explicit Arena(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t n, size_t &off) {
        n = al(std::max<size_t>(n, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            off = it->first;
            const size_t rem = it->second - n;
            free_.erase(it);
            if (rem) free_[off + n] = rem;
            used_ += n;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = al(std::max<size_t>(n, 1));
        used_ -= n;
        auto it = free_.emplace(off, n).first;
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
    size_t size() const { return size_; }
    size_t peak() const { return peak_; }

private:
    size_t size_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

int elem_of(int dt) { return dt == DPM_U8 ? 1 : dt == DPM_U16 ? 2 : 0; }

struct Req {
    dpm_request r;
    double t_arr;
    bool batchable = false;  // the batched path can plan this volume on its own
    size_t bytes() const { return (size_t)(r.dims[0] * r.dims[1] * r.dims[2]) * (size_t)elem_of(r.dtype); }
    int64_t voxels() const { return r.dims[0] * r.dims[1] * r.dims[2]; }
};

struct Block {
    bool host;  // pinned arena or device arena
    size_t off, n;
};

struct Job {
    std::vector<Req> reqs;
    bool batched = false;
    int stream = 0;
    int K = 0;
    hipEvent_t ev = nullptr;
    std::vector<Block> blocks;
    size_t res_off = 0;  // pinned results: exact [n][nm4] then fp64 [n][nm]
    double t_start = 0;
    int status = DPM_OK;
    int nlr = 4;                 // limbs of the 2D moments (resident blocks)
    std::vector<int> keep_bi;    // per request: index in blocks of its resident block, or -1
};

// 2D moments kept on the device after completion: slot-collapsed tiles, order K.
struct Resident {
    size_t off = 0, n = 0;
    int K = 0, nlr = 4;
    uint64_t tick = 0;
};

size_t resident_bytes(int K, int nlr) { return (size_t)2 * (K + 1) * (K + 1) * (K + 1) * nlr * 4; }

// Query scratch allocated at creation: re-strided 2D moments and the outputs.
constexpr size_t kQueryPart = 2 * 17 * 17 * 17 * 12 * 4;
constexpr size_t kQueryOut = 35 * 16 + 969 * 8;

}  // namespace

struct dpm_server {
    dpm_server_config cfg{};
    uint8_t *dev = nullptr;   // device arena
    uint8_t *pin = nullptr;   // pinned result staging
    Arena *darena = nullptr, *parena = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_jobs;

    std::mutex mu;
    std::condition_variable cv_in, cv_out;
    std::deque<Req> incoming;
    std::deque<dpm_completion> done;
    bool stop = false;

    // worker-only state
    std::deque<Req> pending;
    std::vector<Job> inflight;
    std::thread worker;

    // statistics (under mu)
    dpm_server_stats st{};

    // resident 2D moments; the map and the device arena are guarded by res_mu (the worker
    // and the query / release calls of other threads touch them)
    std::mutex res_mu;
    std::map<uint64_t, Resident> resident;
    uint64_t res_tick = 0;
    hipStream_t qstream = nullptr;   // queries
    uint8_t *qdev = nullptr;         // query scratch (device, outside the arena)
    uint8_t *qhost = nullptr;        // pinned query results

    bool evict_one();

    size_t pin_bytes_per_job() const {
        const size_t b = (size_t)cfg.batch_max * (size_t)(dpm::n_moments(4) * 16 + dpm::n_moments(6) * 8);
        const size_t s = (size_t)dpm::n_moments(4) * 16 + (size_t)dpm::n_moments(dpm::KMAX) * 8;
        return al(std::max(b, s));
    }
    bool small(const Req &q) const { return q.batchable && q.voxels() <= cfg.batch_voxels; }

    void release_blocks(Job &j) {
        std::lock_guard<std::mutex> lk(res_mu);
        for (auto &b : j.blocks) (b.host ? parena : darena)->release(b.off, b.n);
        j.blocks.clear();
    }
    bool take(Job &j, bool host, size_t n, size_t &off) {
        std::lock_guard<std::mutex> lk(res_mu);
        if (!(host ? parena : darena)->alloc(n, off)) return false;
        j.blocks.push_back({host, off, n});
        return true;
    }
    // Device blocks a request group needs; false if they do not fit right now.
    bool reserve(Job &j);
    int launch(Job &j);
    void finish(Job &j, int status);
    void run();
};

bool dpm_server::reserve(Job &j) {
    const int n = (int)j.reqs.size();
    const int nm = dpm::n_moments(j.K), nm4 = dpm::n_moments(std::min(j.K, 4));
    size_t off;
    j.keep_bi.assign(n, -1);
    if (!take(j, true, pin_bytes_per_job(), j.res_off)) return false;
    if (j.batched) {
        size_t packed = 0;
        for (auto &q : j.reqs) packed += (q.bytes() + 15) / 16 * 16;
        if (!take(j, false, packed, off)) return false;
        std::vector<dpm_roi> rois(n);
        size_t o = 0;
        for (int i = 0; i < n; ++i) {
            rois[i] = dpm_roi{o, {j.reqs[i].r.dims[0], j.reqs[i].r.dims[1], j.reqs[i].r.dims[2]}, j.reqs[i].r.dtype, 0};
            o += (j.reqs[i].bytes() + 15) / 16 * 16;
        }
        const size_t ws = dpm_batched_workspace_bytes(rois.data(), n, j.K);
        if (!ws || !take(j, false, ws, off)) return false;
        if (!take(j, false, (size_t)n * (nm4 * 16 + nm * 8), off)) return false;
        size_t po, ro;
        if (dpm::batched_partials(rois.data(), n, j.K, 0, &po, &ro, &j.nlr)) return false;
    } else {
        const Req &q = j.reqs[0];
        if (!q.r.data_on_device && !take(j, false, q.bytes(), off)) return false;
        const size_t ws = dpm_workspace_bytes(q.r.dims, (dpm_dtype)q.r.dtype, j.K);
        if (!ws || !take(j, false, ws, off)) return false;
        if (!take(j, false, (size_t)(nm4 * 16 + nm * 8), off)) return false;
        size_t po;
        int32_t t0[dpm::NSLOT + 1];
        if (dpm::single_partials(q.r.dims, (dpm_dtype)q.r.dtype, j.K, &po, t0, &j.nlr)) return false;
    }
    // blocks that stay after completion: the resident 2D moments of kept requests
    for (int i = 0; i < n; ++i)
        if (j.reqs[i].r.keep_resident) {
            if (!take(j, false, resident_bytes(j.K, j.nlr), off)) return false;
            j.keep_bi[i] = (int)j.blocks.size() - 1;
        }
    return true;
}

bool dpm_server::evict_one() {
    std::lock_guard<std::mutex> lk(res_mu);
    if (resident.empty()) return false;
    auto victim = resident.begin();
    for (auto it = resident.begin(); it != resident.end(); ++it)
        if (it->second.tick < victim->second.tick) victim = it;
    darena->release(victim->second.off, victim->second.n);
    resident.erase(victim);
    std::lock_guard<std::mutex> lk2(mu);
    st.evictions += 1;
    st.resident = (int64_t)resident.size();
    int64_t b = 0;
    for (auto &kv : resident) b += (int64_t)kv.second.n;
    st.resident_bytes = b;
    return true;
}

int dpm_server::launch(Job &j) {
    hipStream_t s = streams[j.stream];
    const int n = (int)j.reqs.size();
    const int nm = dpm::n_moments(j.K), nm4 = dpm::n_moments(std::min(j.K, 4));
    j.t_start = now_ms_impl();
    size_t bi = 1;  // blocks[0] is the pinned result staging
    hipError_t e = hipSuccess;
    // device inputs: wait for the work that produces them
    for (auto &q : j.reqs)
        if (q.r.data_on_device && q.r.ready_event) {
            e = hipStreamWaitEvent(s, static_cast<hipEvent_t>(q.r.ready_event), 0);
            if (e != hipSuccess) return DPM_EDEVICE;
        }
    if (j.batched) {
        uint8_t *packed = dev + j.blocks[bi++].off;
        std::vector<dpm_roi> rois(n);
        size_t o = 0;
        for (int i = 0; i < n && e == hipSuccess; ++i) {
            const Req &q = j.reqs[i];
            rois[i] = dpm_roi{o, {q.r.dims[0], q.r.dims[1], q.r.dims[2]}, q.r.dtype, 0};
            e = hipMemcpyAsync(packed + o, q.r.data, q.bytes(),
                               q.r.data_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
            o += (q.bytes() + 15) / 16 * 16;
        }
        if (e != hipSuccess) return DPM_EDEVICE;
        const Block &wb = j.blocks[bi++];
        const Block &ob = j.blocks[bi++];
        dpm_out out{reinterpret_cast<dpm_i128 *>(dev + ob.off),
                    reinterpret_cast<double *>(dev + ob.off + (size_t)n * nm4 * 16)};
        int rc = dpm::batched_run(packed, rois.data(), n, j.K, &out, dev + wb.off, wb.n, s, false);
        if (rc) return rc;
        for (int i = 0; i < n && e == hipSuccess; ++i) {
            if (j.keep_bi[i] < 0) continue;
            size_t po, ro;
            int nlr;
            if ((rc = dpm::batched_partials(rois.data(), n, j.K, i, &po, &ro, &nlr))) return rc;
            dpm::CollapseArgs c{};
            c.part = reinterpret_cast<const uint32_t *>(dev + wb.off + po);
            c.roi = reinterpret_cast<const dpm::RoiDesc *>(dev + wb.off + ro);
            c.K = j.K;
            c.nlr = nlr;
            c.out = reinterpret_cast<uint32_t *>(dev + j.blocks[j.keep_bi[i]].off);
            e = dpm::launch_collapse(c, s);
        }
        if (e != hipSuccess) return DPM_EDEVICE;
        e = hipMemcpyAsync(pin + j.res_off, dev + ob.off, (size_t)n * (nm4 * 16 + nm * 8), hipMemcpyDeviceToHost, s);
    } else {
        const Req &q = j.reqs[0];
        const void *vol = q.r.data;
        if (!q.r.data_on_device) {
            uint8_t *v = dev + j.blocks[bi++].off;
            e = hipMemcpyAsync(v, q.r.data, q.bytes(), hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return DPM_EDEVICE;
            vol = v;
        }
        const Block &wb = j.blocks[bi++];
        const Block &ob = j.blocks[bi++];
        dpm_out out{reinterpret_cast<dpm_i128 *>(dev + ob.off), reinterpret_cast<double *>(dev + ob.off + nm4 * 16)};
        int rc = dpm_moments_async(vol, q.r.dims, (dpm_dtype)q.r.dtype, j.K, &out, dev + wb.off, wb.n, s);
        if (rc) return rc;
        if (j.keep_bi[0] >= 0) {
            dpm::CollapseArgs c{};
            size_t po;
            if ((rc = dpm::single_partials(q.r.dims, (dpm_dtype)q.r.dtype, j.K, &po, c.tile0, &c.nlr))) return rc;
            c.part = reinterpret_cast<const uint32_t *>(dev + wb.off + po);
            c.roi = nullptr;
            c.K = j.K;
            c.out = reinterpret_cast<uint32_t *>(dev + j.blocks[j.keep_bi[0]].off);
            if (dpm::launch_collapse(c, s) != hipSuccess) return DPM_EDEVICE;
        }
        e = hipMemcpyAsync(pin + j.res_off, dev + ob.off, (size_t)(nm4 * 16 + nm * 8), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipEventRecord(j.ev, s);
    return e == hipSuccess ? DPM_OK : DPM_EDEVICE;
}

void dpm_server::finish(Job &j, int status) {
    const int n = (int)j.reqs.size();
    const int nm = dpm::n_moments(j.K), nm4 = dpm::n_moments(std::min(j.K, 4));
    const uint8_t *res = pin + j.res_off;
    std::vector<dpm_completion> out;
    for (int i = 0; i < n; ++i) {
        const Req &q = j.reqs[i];
        if (status == DPM_OK) {
            // graded order: the moments of order <= K_request are a prefix of the job's
            const int k = q.r.max_order;
            if (q.r.exact)
                std::memcpy(q.r.exact, res + (size_t)i * nm4 * 16, (size_t)dpm::n_moments(std::min(k, 4)) * 16);
            if (q.r.fp64)
                std::memcpy(q.r.fp64, res + (size_t)n * nm4 * 16 + (size_t)i * nm * 8, (size_t)dpm::n_moments(k) * 8);
        }
        out.push_back(dpm_completion{q.r.tag, status, j.batched ? 1 : 0, q.t_arr, j.t_start, now_ms_impl()});
    }
    if (status == DPM_OK) {
        // kept requests: their resident blocks leave the job (released on eviction)
        std::vector<bool> kept(j.blocks.size(), false);
        {
            std::lock_guard<std::mutex> lk(res_mu);
            for (int i = 0; i < n; ++i) {
                if (j.keep_bi.size() != (size_t)n || j.keep_bi[i] < 0) continue;
                const Block &b = j.blocks[j.keep_bi[i]];
                auto old = resident.find(j.reqs[i].r.tag);
                if (old != resident.end()) {
                    darena->release(old->second.off, old->second.n);
                    resident.erase(old);
                }
                resident[j.reqs[i].r.tag] = Resident{b.off, b.n, j.K, j.nlr, ++res_tick};
                kept[j.keep_bi[i]] = true;
            }
            int64_t bytes = 0;
            for (auto &kv : resident) bytes += (int64_t)kv.second.n;
            std::lock_guard<std::mutex> lk2(mu);
            st.resident = (int64_t)resident.size();
            st.resident_bytes = bytes;
        }
        std::vector<Block> rest;
        for (size_t b = 0; b < j.blocks.size(); ++b)
            if (!kept[b]) rest.push_back(j.blocks[b]);
        j.blocks.swap(rest);
    }
    release_blocks(j);
    stream_jobs[j.stream]--;
    std::lock_guard<std::mutex> lk(mu);
    for (auto &c : out) done.push_back(c);
    st.completed += n;
    (j.batched ? st.batched_jobs : st.single_jobs) += 1;
    st.arena_peak_used = (int64_t)darena->peak();
    cv_out.notify_all();
}

void dpm_server::run() {
    (void)hipSetDevice(cfg.device);
    std::vector<hipEvent_t> free_events;
    for (;;) {
        bool stopping;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (incoming.empty() && inflight.empty() && pending.empty() && !stop)
                cv_in.wait(lk, [&] { return stop || !incoming.empty(); });
            while (!incoming.empty()) {
                pending.push_back(incoming.front());
                incoming.pop_front();
            }
            stopping = stop;
            st.pending = (int32_t)pending.size();
            st.inflight = (int32_t)inflight.size();
        }
        // retire finished jobs
        for (size_t i = 0; i < inflight.size();) {
            hipError_t q = hipEventQuery(inflight[i].ev);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            finish(inflight[i], q == hipSuccess ? DPM_OK : DPM_EDEVICE);
            free_events.push_back(inflight[i].ev);
            inflight.erase(inflight.begin() + (long)i);
        }
        // admit first come, first served
        while (!pending.empty() && (int)inflight.size() < cfg.max_inflight) {
            Job j;
            if (small(pending.front())) {
                j.batched = true;
                // continuous batching: every waiting small request of the same order as the
                // first, in arrival order (a batch runs at one order)
                const int kb = pending.front().r.max_order;
                for (auto it = pending.begin(); it != pending.end() && (int)j.reqs.size() < cfg.batch_max;) {
                    if (small(*it) && it->r.max_order == kb) {
                        j.reqs.push_back(*it);
                        it = pending.erase(it);
                    } else {
                        ++it;
                    }
                }
            } else {
                j.reqs.push_back(pending.front());
                pending.pop_front();
            }
            for (auto &q : j.reqs) j.K = std::max(j.K, q.r.max_order);
            bool ok = reserve(j);
            while (!ok) {
                // make room: drop resident 2D moments, least recently used first
                release_blocks(j);
                if (!evict_one()) break;
                ok = reserve(j);
            }
            if (!ok) {
                // does not fit now: put the group back at the front, in order
                release_blocks(j);
                for (auto it = j.reqs.rbegin(); it != j.reqs.rend(); ++it) pending.push_front(*it);
                if (!inflight.empty()) break;
                // nothing in flight and still no room: the group is too large together;
                // serve its first request alone
                Job one;
                one.reqs.push_back(pending.front());
                pending.pop_front();
                one.K = one.reqs[0].r.max_order;
                one.batched = small(one.reqs[0]);
                bool ok1 = reserve(one);
                while (!ok1) {
                    release_blocks(one);
                    if (!evict_one()) break;
                    ok1 = reserve(one);
                }
                if (!ok1) {
                    release_blocks(one);
                    stream_jobs[one.stream]++;  // finish() releases one job of its stream
                    finish(one, DPM_ENOMEM);
                    continue;
                }
                j = std::move(one);
            }
            int best = 0;
            for (int s = 1; s < (int)streams.size(); ++s)
                if (stream_jobs[s] < stream_jobs[best]) best = s;
            j.stream = best;
            stream_jobs[best]++;
            if (free_events.empty()) {
                hipEvent_t ev;
                if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                    finish(j, DPM_EDEVICE);  // releases its blocks and its stream count
                    continue;
                }
                free_events.push_back(ev);
            }
            j.ev = free_events.back();
            free_events.pop_back();
            int rc = launch(j);
            if (rc) {
                // the stream may hold part of the job: wait for it before freeing blocks
                (void)hipStreamSynchronize(streams[j.stream]);
                free_events.push_back(j.ev);
                finish(j, rc);
                continue;
            }
            inflight.push_back(std::move(j));
        }
        if (stopping && pending.empty() && inflight.empty()) break;
        if (!inflight.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    for (auto ev : free_events) (void)hipEventDestroy(ev);
}

extern "C" {

double dpm_server_now_ms(void) { return now_ms_impl(); }

int dpm_server_create(const dpm_server_config *cfg, dpm_server **out) {
    if (!cfg || !out || cfg->n_streams < 1 || cfg->hbm_budget <= 0 || cfg->batch_max < 1 || cfg->max_inflight < 1)
        return DPM_EINVAL;
    *out = nullptr;
    auto *s = new dpm_server();
    s->cfg = *cfg;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (hipSetDevice(cfg->device) != hipSuccess) {
        delete s;
        return DPM_EINVAL;
    }
    const size_t pbytes = (size_t)cfg->max_inflight * s->pin_bytes_per_job();
    bool ok = hipMalloc(reinterpret_cast<void **>(&s->dev), (size_t)cfg->hbm_budget) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void **>(&s->pin), pbytes, hipHostMallocDefault) == hipSuccess;
    for (int i = 0; ok && i < cfg->n_streams; ++i) {
        hipStream_t st;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;  // default priority
        if (ok) s->streams.push_back(st);
    }
    ok = ok && hipStreamCreateWithFlags(&s->qstream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipHostMalloc(reinterpret_cast<void **>(&s->qhost), kQueryOut, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void **>(&s->qdev), kQueryPart + kQueryOut) == hipSuccess;
    // warm every stream before serving: its first dispatch binds it to a hardware queue,
    // which would otherwise delay the first requests by milliseconds
    for (size_t i = 0; ok && i < s->streams.size(); ++i)
        ok = hipMemsetAsync(s->dev, 0, 256, s->streams[i]) == hipSuccess && hipStreamSynchronize(s->streams[i]) == hipSuccess;
    ok = ok && hipMemsetAsync(s->dev, 0, 256, s->qstream) == hipSuccess && hipStreamSynchronize(s->qstream) == hipSuccess;
    (void)hipSetDevice(cur);
    if (!ok) {
        for (auto st : s->streams) (void)hipStreamDestroy(st);
        if (s->qstream) (void)hipStreamDestroy(s->qstream);
        if (s->dev) (void)hipFree(s->dev);
        if (s->pin) (void)hipHostFree(s->pin);
        if (s->qhost) (void)hipHostFree(s->qhost);
        if (s->qdev) (void)hipFree(s->qdev);
        delete s;
        return DPM_ENOMEM;
    }
    s->darena = new Arena((size_t)cfg->hbm_budget);
    s->parena = new Arena(pbytes);
    s->stream_jobs.assign(cfg->n_streams, 0);
    s->st.arena_bytes = cfg->hbm_budget;
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return DPM_OK;
}

int dpm_server_submit(dpm_server *s, const dpm_request *req) {
    if (!s || !req || !req->data || req->max_order < 0 || req->max_order > dpm::KMAX || !elem_of(req->dtype) ||
        req->dims[0] <= 0 || req->dims[1] <= 0 || req->dims[2] <= 0)
        return DPM_EINVAL;
    Req q{*req, req->t_arrival_ms > 0 ? req->t_arrival_ms : now_ms_impl()};
    if (req->max_order <= 6 && req->dims[0] <= 4096 && req->dims[1] <= 4096 && req->dims[2] <= 4096) {
        // batchable if the batched planner accepts it alone (then also in any batch:
        // a batch plan takes the maximum of its ROIs' widths and LDS)
        dpm_roi roi{};
        roi.dims[0] = req->dims[0];
        roi.dims[1] = req->dims[1];
        roi.dims[2] = req->dims[2];
        roi.dtype = req->dtype;
        q.batchable = dpm_batched_workspace_bytes(&roi, 1, req->max_order) > 0;
    }
    // refuse what can never fit: its own blocks exceed the whole arena
    const size_t ws = dpm_workspace_bytes(req->dims, (dpm_dtype)req->dtype, req->max_order);
    if (!ws) return DPM_ERANGE;
    const size_t need = al(ws) + al(req->data_on_device ? 0 : q.bytes()) + al(16 * 1024) +
                        (req->keep_resident ? al(resident_bytes(req->max_order, 12)) : 0);
    if (need > (size_t)s->cfg.hbm_budget) return DPM_ERANGE;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return DPM_EINVAL;
        s->incoming.push_back(q);
        s->st.submitted += 1;
    }
    s->cv_in.notify_one();
    return DPM_OK;
}

int dpm_server_poll(dpm_server *s, dpm_completion *out, int max, int wait_ms) {
    if (!s || (!out && max > 0) || max < 0) return DPM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_ms > 0)
        s->cv_out.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
    int n = 0;
    while (n < max && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    return n;
}

int dpm_server_replay(dpm_server *s, const dpm_request *reqs, int n) {
    if (!s || (!reqs && n > 0) || n < 0) return DPM_EINVAL;
    for (int i = 0; i < n; ++i) {
        const double t = reqs[i].t_arrival_ms;
        for (;;) {
            const double left = t - now_ms_impl();
            if (left <= 0) break;
            if (left > 0.2) std::this_thread::sleep_for(std::chrono::microseconds((int64_t)((left - 0.2) * 1000)));
        }
        const int rc = dpm_server_submit(s, &reqs[i]);
        if (rc) return rc;
    }
    return DPM_OK;
}

int dpm_server_requery(dpm_server *s, uint64_t tag, int max_order, dpm_i128 *exact, double *fp64) {
    if (!s || max_order < 0 || max_order > dpm::KMAX) return DPM_EINVAL;
    std::lock_guard<std::mutex> lk(s->res_mu);
    auto it = s->resident.find(tag);
    if (it == s->resident.end() || max_order > it->second.K) return DPM_EINVAL;
    Resident &r = it->second;
    r.tick = ++s->res_tick;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (hipSetDevice(s->cfg.device) != hipSuccess) return DPM_EDEVICE;
    int rc = dpm::batched_ensure_tables();
    const int K = max_order, nm = dpm::n_moments(K), nm4 = dpm::n_moments(std::min(K, 4));
    uint8_t *qpart = s->qdev, *qout = qpart + kQueryPart;
    const uint32_t *part = reinterpret_cast<const uint32_t *>(s->dev + r.off);
    hipError_t e = hipSuccess;
    if (!rc && K < r.K) {
        // the recombination reads tiles laid out for its own order: re-stride first
        e = dpm::launch_restride(part, r.K, reinterpret_cast<uint32_t *>(qpart), K, r.nlr, s->qstream);
        part = reinterpret_cast<const uint32_t *>(qpart);
    }
    if (!rc && e == hipSuccess) {
        // one tile per image side: tile s holds slot s (Section 3.2 recombination)
        dpm::FinishArgs f{};
        f.part = part;
        f.rois = nullptr;
        f.nvol = 1;
        f.K = K;
        for (int sl = 0; sl <= dpm::NSLOT; ++sl) f.tile0[sl] = std::min(sl, 2 * (K + 1));
        f.exact = qout;
        f.fp64 = reinterpret_cast<double *>(qout + 35 * 16);
        f.raw = nullptr;
        e = dpm::launch_finish(r.nlr, f, s->qstream);
    }
    if (!rc && e == hipSuccess) e = hipMemcpyAsync(s->qhost, qout, kQueryOut, hipMemcpyDeviceToHost, s->qstream);
    if (!rc && e == hipSuccess) e = hipStreamSynchronize(s->qstream);
    (void)hipSetDevice(cur);
    if (rc) return rc;
    if (e != hipSuccess) return DPM_EDEVICE;
    if (exact) std::memcpy(exact, s->qhost, (size_t)nm4 * 16);
    if (fp64) std::memcpy(fp64, s->qhost + 35 * 16, (size_t)nm * 8);
    return DPM_OK;
}

int dpm_server_release(dpm_server *s, uint64_t tag) {
    if (!s) return DPM_EINVAL;
    std::lock_guard<std::mutex> lk(s->res_mu);
    auto it = s->resident.find(tag);
    if (it == s->resident.end()) return DPM_EINVAL;
    s->darena->release(it->second.off, it->second.n);
    s->resident.erase(it);
    int64_t b = 0;
    for (auto &kv : s->resident) b += (int64_t)kv.second.n;
    std::lock_guard<std::mutex> lk2(s->mu);
    s->st.resident = (int64_t)s->resident.size();
    s->st.resident_bytes = b;
    return DPM_OK;
}

int dpm_server_stats_get(dpm_server *s, dpm_server_stats *out) {
    if (!s || !out) return DPM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    return DPM_OK;
}

int dpm_server_destroy(dpm_server *s) {
    if (!s) return DPM_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_in.notify_all();
    if (s->worker.joinable()) s->worker.join();
    int rc = DPM_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(s->cfg.device);
    for (auto st : s->streams)
        if (hipStreamDestroy(st) != hipSuccess) rc = DPM_EDEVICE;
    if (s->qstream && hipStreamDestroy(s->qstream) != hipSuccess) rc = DPM_EDEVICE;
    if (s->dev && hipFree(s->dev) != hipSuccess) rc = DPM_EDEVICE;
    if (s->pin && hipHostFree(s->pin) != hipSuccess) rc = DPM_EDEVICE;
    if (s->qhost && hipHostFree(s->qhost) != hipSuccess) rc = DPM_EDEVICE;
    if (s->qdev && hipFree(s->qdev) != hipSuccess) rc = DPM_EDEVICE;
    (void)hipSetDevice(cur);
    delete s->darena;
    delete s->parena;
    delete s;
    return rc;
}

}  // extern "C"
