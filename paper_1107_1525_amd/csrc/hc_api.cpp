// C ABI entry points: argument checks, then kernel launches on the caller's
// stream.  See include/hc.h for the contract of every call.
#include <hip/hip_runtime_api.h>
#include <sched.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "hc_internal.h"
#include "hc_kernels.h"

using namespace hc;

namespace {

// Launch parameters the autotuner may set (hc_set_tuning): the most 16-byte
// loads per thread of an encode tile (0: the library's rule alone).
std::atomic<uint32_t> g_tile_loads_cap{0};

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

bool valid_block_size(uint32_t B) { return B >= 16 && B <= (1u << 26) && (B % 16) == 0; }

bool valid_sub_block(uint32_t S) { return S == 0 || (S % 16) == 0; }

hc_status hip_status(hipError_t e) { return e == hipSuccess ? HC_OK : HC_ERR_HIP; }

// A parallel for over [0, count) on a few host threads, the caller included,
// for the per-stream code builds of a codebook set (independent, a few
// microseconds each, and on the critical path between the counting and the
// encoding kernels).  The workers live for the process (a forked child makes
// its own); one loop runs at a time.
class HostPool {
public:
    static HostPool &get()
    {
        static std::mutex m;
        static HostPool *pool = nullptr;
        std::lock_guard<std::mutex> g(m);
        if (!pool || pool->pid_ != getpid()) pool = new HostPool();  // a forked child's workers did not survive
        return *pool;
    }

    void run(uint32_t count, const std::function<void(uint32_t)> &f)
    {
        std::lock_guard<std::mutex> one_at_a_time(run_m_);
        if (workers_ == 0 || count < 4) {
            for (uint32_t i = 0; i < count; ++i) f(i);
            return;
        }
        {
            std::lock_guard<std::mutex> g(m_);
            f_ = &f;
            count_ = count;
            next_.store(0);
            busy_ = workers_;
            ++generation_;
        }
        cv_.notify_all();
        drain();
        std::unique_lock<std::mutex> g(m_);
        done_cv_.wait(g, [&] { return busy_ == 0; });
        f_ = nullptr;
    }

private:
    HostPool() : pid_(getpid())
    {
        cpu_set_t set;
        unsigned cpus = std::thread::hardware_concurrency();
        if (sched_getaffinity(0, sizeof(set), &set) == 0) cpus = (unsigned)CPU_COUNT(&set);
        workers_ = cpus > 1 ? std::min(cpus - 1, 7u) : 0u;
        for (unsigned w = 0; w < workers_; ++w) std::thread([this] { loop(); }).detach();
    }

    void drain()
    {
        for (uint32_t i = next_.fetch_add(1); i < count_; i = next_.fetch_add(1)) (*f_)(i);
    }

    void loop()
    {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> g(m_);
                cv_.wait(g, [&] { return generation_ != seen; });
                seen = generation_;
            }
            drain();
            std::lock_guard<std::mutex> g(m_);
            if (--busy_ == 0) done_cv_.notify_one();
        }
    }

    pid_t pid_;
    unsigned workers_ = 0;
    std::mutex run_m_, m_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(uint32_t)> *f_ = nullptr;
    uint32_t count_ = 0;
    std::atomic<uint32_t> next_{0};
    unsigned busy_ = 0;
    uint64_t generation_ = 0;
};

}  // namespace

extern "C" const char *hc_status_str(int status)
{
    switch (status) {
    case HC_OK: return "HC_OK";
    case HC_ERR_INVALID_ARG: return "HC_ERR_INVALID_ARG";
    case HC_ERR_NO_SPACE: return "HC_ERR_NO_SPACE";
    case HC_ERR_HIP: return "HC_ERR_HIP";
    case HC_ERR_SYMBOL_ABSENT: return "HC_ERR_SYMBOL_ABSENT";
    case HC_ERR_BLOCK_OVERFLOW: return "HC_ERR_BLOCK_OVERFLOW";
    case HC_ERR_CORRUPT: return "HC_ERR_CORRUPT";
    case HC_ERR_CODE_TOO_LONG: return "HC_ERR_CODE_TOO_LONG";
    case HC_ERR_TABLE_CHANGED: return "HC_ERR_TABLE_CHANGED";
    default: return "HC_ERR_UNKNOWN";
    }
}

extern "C" int hc_version(void) { return 100; }

extern "C" hc_status hc_set_tuning(const hc_tuning *t)
{
    if (!t) return HC_ERR_INVALID_ARG;
    const uint32_t q = t->encode_tile_loads;
    if (q != 0 && q != 1 && q != 2 && q != 4) return HC_ERR_INVALID_ARG;
    g_tile_loads_cap.store(q, std::memory_order_relaxed);
    return HC_OK;
}

extern "C" hc_status hc_get_tuning(hc_tuning *t)
{
    if (!t) return HC_ERR_INVALID_ARG;
    t->encode_tile_loads = g_tile_loads_cap.load(std::memory_order_relaxed);
    return HC_OK;
}

namespace {

// The codebook must be the canonical code of its own lengths.
hc_status validate_codebook(const hc_codebook *cb)
{
    hc_codebook check;
    hc_status st = canonical_from_lengths(cb->len, &check);
    if (st != HC_OK) return st;
    if (check.max_len != cb->max_len || check.nsym != cb->nsym ||
        memcmp(check.code, cb->code, sizeof(check.code)) != 0)
        return HC_ERR_INVALID_ARG;
    return HC_OK;
}

void release(hc_cb_dev_s *h)
{
    if (h->d_tables) (void)hipFree(h->d_tables);
    if (h->staging) (void)hipHostFree(h->staging);
    if (h->copy_done) (void)hipEventDestroy(static_cast<hipEvent_t>(h->copy_done));
    free(h);
}

}  // namespace

extern "C" hc_status hc_codebook_upload(const hc_codebook *cb, hc_cb_handle *out)
{
    if (!cb || !out) return HC_ERR_INVALID_ARG;
    *out = nullptr;
    hc_status st = validate_codebook(cb);
    if (st != HC_OK) return st;
    hc_cb_dev_s *h = static_cast<hc_cb_dev_s *>(calloc(1, sizeof(hc_cb_dev_s)));
    if (!h) return HC_ERR_INVALID_ARG;
    h->host = *cb;
    hipEvent_t ev = nullptr;
    if (hipGetDevice(&h->device) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&h->staging), sizeof(DevTables), hipHostMallocDefault) !=
            hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&h->d_tables), sizeof(DevTables)) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        release(h);
        return HC_ERR_HIP;
    }
    h->copy_done = ev;
    build_dev_tables(*cb, h->staging);
    if (hipMemcpy(h->d_tables, h->staging, sizeof(DevTables), hipMemcpyHostToDevice) != hipSuccess) {
        release(h);
        return HC_ERR_HIP;
    }
    *out = h;
    return HC_OK;
}

extern "C" hc_status hc_codebook_update(hc_cb_handle h, const hc_codebook *cb, void *stream)
{
    if (!h || !cb || h->in_set) return HC_ERR_INVALID_ARG;
    hc_status st = validate_codebook(cb);
    if (st != HC_OK) return st;
    hipEvent_t ev = static_cast<hipEvent_t>(h->copy_done);
    if (hipEventSynchronize(ev) != hipSuccess) return HC_ERR_HIP;  // staging no longer being read
    build_dev_tables(*cb, h->staging);
    h->host = *cb;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(h->d_tables, h->staging, sizeof(DevTables), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(ev, s) != hipSuccess)
        return HC_ERR_HIP;
    return HC_OK;
}

extern "C" hc_status hc_cbset_create(uint32_t count, hc_cbset *out)
{
    if (!out || count == 0) return HC_ERR_INVALID_ARG;
    *out = nullptr;
    hc_cbset_s *set = static_cast<hc_cbset_s *>(calloc(1, sizeof(hc_cbset_s)));
    if (!set) return HC_ERR_INVALID_ARG;
    set->count = count;
    set->handles = static_cast<hc_cb_dev_s *>(calloc(count, sizeof(hc_cb_dev_s)));
    hipEvent_t ev = nullptr;
    int dev = 0;
    const size_t bytes = (size_t)count * sizeof(DevTables);
    if (!set->handles || hipGetDevice(&dev) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&set->staging), bytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&set->d_tables), bytes) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        if (set->d_tables) (void)hipFree(set->d_tables);
        if (set->staging) (void)hipHostFree(set->staging);
        free(set->handles);
        free(set);
        return HC_ERR_HIP;
    }
    set->copy_done = ev;
    // Until the first build every table is the empty code (no symbol has a code).
    memset(set->staging, 0, bytes);
    for (uint32_t k = 0; k < count; ++k) {
        hc_cb_dev_s &h = set->handles[k];
        build_dev_tables(h.host, &set->staging[k]);
        h.d_tables = &set->d_tables[k];
        h.device = dev;
        h.in_set = 1;
    }
    if (hipMemcpy(set->d_tables, set->staging, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(set->d_tables);
        (void)hipHostFree(set->staging);
        (void)hipEventDestroy(ev);
        free(set->handles);
        free(set);
        return HC_ERR_HIP;
    }
    *out = set;
    return HC_OK;
}

extern "C" hc_cb_handle hc_cbset_handle(hc_cbset set, uint32_t k)
{
    if (!set || k >= set->count) return nullptr;
    return &set->handles[k];
}

extern "C" hc_status hc_cbset_build(hc_cbset set, const uint64_t *h_hists, hc_codebook *h_out, void *stream)
{
    if (!set || !h_hists) return HC_ERR_INVALID_ARG;
    hipEvent_t ev = static_cast<hipEvent_t>(set->copy_done);
    if (hipEventSynchronize(ev) != hipSuccess) return HC_ERR_HIP;  // staging no longer being read
    // the codes of the set's streams are independent: built on several host threads
    std::atomic<int> first_error{HC_OK};
    HostPool::get().run(set->count, [&](uint32_t k) {
        hc_codebook cb;
        hc_status st = hc_build_codebook(h_hists + (size_t)256 * k, &cb);
        if (st != HC_OK) {
            int ok = HC_OK;
            first_error.compare_exchange_strong(ok, st);
            return;
        }
        if (cb.max_len == 0) {  // an empty buffer: a one-symbol code keeps the tables usable
            uint8_t len[kNumSym] = {0};
            len[0] = 1;
            canonical_from_lengths(len, &cb);
        }
        set->handles[k].host = cb;
        build_dev_tables(cb, &set->staging[k]);
        if (h_out) h_out[k] = cb;
    });
    if (first_error.load() != HC_OK) return static_cast<hc_status>(first_error.load());
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(set->d_tables, set->staging, (size_t)set->count * sizeof(DevTables), hipMemcpyHostToDevice,
                       s) != hipSuccess ||
        hipEventRecord(ev, s) != hipSuccess)
        return HC_ERR_HIP;
    return HC_OK;
}

extern "C" hc_status hc_cbset_destroy(hc_cbset set)
{
    if (!set) return HC_OK;
    // the set's own last copy out of its staging area; launches reading the
    // tables are the caller's to have ordered before this call
    hipError_t e = hipEventSynchronize(static_cast<hipEvent_t>(set->copy_done));
    (void)hipFree(set->d_tables);
    (void)hipHostFree(set->staging);
    (void)hipEventDestroy(static_cast<hipEvent_t>(set->copy_done));
    free(set->handles);
    free(set);
    return hip_status(e);
}

extern "C" hc_status hc_codebook_destroy(hc_cb_handle cb)
{
    if (!cb || cb->in_set) return HC_OK;
    // the handle's own last table copy; launches reading it are the caller's
    // to have ordered before this call
    hipError_t e = hipEventSynchronize(static_cast<hipEvent_t>(cb->copy_done));
    release(cb);
    return hip_status(e);
}

extern "C" uint64_t hc_encode_bound(uint64_t n, uint32_t block_size, uint32_t max_len)
{
    if (block_size == 0 || max_len > (uint32_t)kMaxLen) return 0;
    const uint64_t full = n / block_size, rest = n % block_size;
    const uint64_t per_full = 4 + 4 * (((uint64_t)block_size * max_len + 31) / 32);
    uint64_t total = full * per_full;
    if (rest) total += 4 + 4 * ((rest * max_len + 31) / 32);
    return total;
}

extern "C" uint64_t hc_encode_workspace_bytes(uint64_t n, uint32_t block_size)
{
    if (block_size == 0) return 0;
    const uint64_t nb = num_blocks(n, block_size);
    return encode_scratch_bound(nb, block_size);
}

extern "C" uint64_t hc_sub_index_entries(uint64_t n, uint32_t block_size, uint32_t sub_block)
{
    if (block_size == 0 || sub_block == 0) return 0;
    return num_blocks(n, block_size) * ((block_size + sub_block - 1) / sub_block);
}

namespace {

// The encode tile shape for B and a longest code: the rule of encode_qpt,
// capped by the tuning (to 1, 2 or 4 loads per thread).
uint32_t tuned_qpt(uint32_t B, uint32_t max_len)
{
    uint32_t q = encode_qpt(B, max_len);
    const uint32_t cap = g_tile_loads_cap.load(std::memory_order_relaxed);
    while (cap && q > cap) q >>= 1;
    return q;
}

Job empty_job()
{
    Job j;
    memset(&j, 0, sizeof(j));
    return j;
}

JobList single(const Job &j)
{
    JobList jl;
    jl.jobs = nullptr;
    jl.starts = nullptr;
    jl.count = 1;
    jl.one = j;
    return jl;
}

// Work-groups of a decode launch: one lane per chunk (decode_chunk symbols).
uint64_t decode_groups(uint64_t n, uint32_t B, uint32_t S, bool with_index, bool complete8)
{
    const uint32_t chunk = decode_chunk(B, S, with_index, complete8);
    const uint64_t lanes = num_blocks(n, B) * ((B + chunk - 1) / chunk);
    return (lanes + kDecThreads - 1) / kDecThreads;
}

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Checks of one encode input; the same for the single and the batched call.
hc_status check_encode(const uint8_t *in, uint64_t n, uint32_t B, hc_cb_handle cb, const uint8_t *out,
                       uint64_t out_cap, const uint64_t *block_off, const uint32_t *sub_idx, uint32_t S)
{
    if (!cb || !block_off || !aligned(block_off, 8)) return HC_ERR_INVALID_ARG;
    if ((sub_idx == nullptr) != (S == 0)) return HC_ERR_INVALID_ARG;
    if (sub_idx && !aligned(sub_idx, 4)) return HC_ERR_INVALID_ARG;
    if (n > 0) {
        if (!in || !aligned(in, 16) || !out || !aligned(out, 16)) return HC_ERR_INVALID_ARG;
        if (cb->host.max_len == 0) return HC_ERR_INVALID_ARG;  // no code for any symbol
        if (out_cap < hc_encode_bound(n, B, cb->host.max_len)) return HC_ERR_NO_SPACE;
    }
    return HC_OK;
}

hc_status check_decode(const uint8_t *in, uint64_t in_bytes, uint64_t n, hc_cb_handle cb, const uint64_t *block_off,
                       const uint32_t *sub_idx, uint32_t S, const uint8_t *out)
{
    if (!cb) return HC_ERR_INVALID_ARG;
    if ((sub_idx == nullptr) != (S == 0)) return HC_ERR_INVALID_ARG;
    if (n == 0) return HC_OK;
    if (!in || !aligned(in, 16) || (in_bytes & 3) || !block_off || !aligned(block_off, 8) || !out ||
        !aligned(out, 16) || (sub_idx && !aligned(sub_idx, 4)))
        return HC_ERR_INVALID_ARG;
    if (cb->host.max_len == 0) return HC_ERR_INVALID_ARG;
    return HC_OK;
}

// Bytes at the head of a batch workspace: the job table, then the start unit
// of every job and the total.
uint64_t job_table_bytes(uint32_t count)
{
    // + room for the alignment of the other tables: the encode and the decode
    // split their jobs into launches by code length, each with its own table
    return align256((uint64_t)count * sizeof(Job)) + align256(8 * ((uint64_t)count + 1)) + 4096;
}

// A complete 8-bit code: all 256 bytes coded, none longer than 8 bits, so
// (Kraft) every code has 8 bits and decoding is a byte-swapped copy.
bool complete8(const hc_codebook &cb) { return cb.max_len == 8 && cb.nsym == 256; }

// Pinned host staging for job tables: a small ring of buffers, each with the
// event of its last copy, so that a table travels to the device as one
// asynchronous copy and the host never waits for the stream (a copy from
// pageable memory would).  A slot is reused only once its previous copy has
// left it (normally long before: eight batch calls ago); a buffer grows when
// a table outgrows it.
class JobStaging {
public:
    static JobStaging &get()
    {
        static JobStaging st;
        return st;
    }
    // Copies 'bytes' of 'fill' output to d_dst on s; returns a HIP error or hipSuccess.
    template <typename Fill>
    hipError_t copy(void *d_dst, size_t bytes, hipStream_t s, const Fill &fill)
    {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        std::lock_guard<std::mutex> g(mu_);
        Slot &sl = slots_[next_++ % kSlots];
        if (sl.ev) {
            e = hipEventSynchronize(sl.ev);  // its previous copy has left the buffer
            if (e != hipSuccess) return e;
        }
        if (sl.dev != dev && sl.ev) {  // events and pinned buffers are made per device
            (void)hipEventDestroy(sl.ev);
            sl.ev = nullptr;
        }
        if (!sl.ev && (e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming)) != hipSuccess) return e;
        sl.dev = dev;
        if (sl.cap < bytes) {
            if (sl.host) (void)hipHostFree(sl.host);
            sl.host = nullptr;
            sl.cap = 0;
            size_t cap = 64 << 10;
            while (cap < bytes) cap *= 2;
            if ((e = hipHostMalloc(&sl.host, cap, hipHostMallocDefault)) != hipSuccess) return e;
            sl.cap = cap;
        }
        fill(static_cast<char *>(sl.host));
        if ((e = hipMemcpyAsync(d_dst, sl.host, bytes, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
        return hipEventRecord(sl.ev, s);
    }

private:
    static constexpr int kSlots = 8;
    struct Slot {
        void *host = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        int dev = -1;
    };
    std::mutex mu_;
    Slot slots_[kSlots];
    uint64_t next_ = 0;
};

// Side by side launches of one call's classes.  A batch call's code classes
// are independent launches; in stream order a memory-bound one (the copy of
// complete 8-bit codes) and a latency-bound one (the table decoder, the
// packing of short codes) leave each other's idle resources unused.  Fork
// hands the caller's stream and up to kSideStreams library-owned streams
// (non-blocking, default priority, one set per device, created on first
// use) that wait for all the caller's stream holds; join makes the caller's
// stream wait for all of them again, so the call stays one step in the
// caller's stream order.  Not used while the stream is captured into a
// graph (a forked stream would stay in the capture): the launches then run
// in stream order.  One call forks at a time (the events are shared).
class SideStreams {
public:
    static constexpr int kSideStreams = 3;

    static SideStreams &get()
    {
        static SideStreams st;
        return st;
    }

    // Streams for 'want' launches: out[0] = s, out[1..] side streams (fewer
    // when s is being captured or on any error: then every entry is s).
    // Holds the fork lock until join.
    void fork(hipStream_t s, int want, hipStream_t *out)
    {
        for (int k = 0; k < want; ++k) out[k] = s;
        forked_ = 0;
        mu_.lock();
        if (want < 2) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return;
        Dev &d = dev_[dev];
        if (!d.ready) {
            for (int k = 0; k < kSideStreams; ++k)
                if (hipStreamCreateWithFlags(&d.side[k], hipStreamNonBlocking) != hipSuccess ||
                    hipEventCreateWithFlags(&d.joined[k], hipEventDisableTiming) != hipSuccess)
                    return;
            if (hipEventCreateWithFlags(&d.start, hipEventDisableTiming) != hipSuccess) return;
            d.ready = true;
        }
        if (hipEventRecord(d.start, s) != hipSuccess) return;
        const int n = want - 1 < kSideStreams ? want - 1 : kSideStreams;
        for (int k = 0; k < n; ++k) {
            if (hipStreamWaitEvent(d.side[k], d.start, 0) != hipSuccess) break;
            forked_ = k + 1;
        }
        cur_ = &d;
        for (int k = 1; k < want; ++k) out[k] = forked_ ? d.side[(k - 1) % forked_] : s;
    }

    // The caller's stream waits for every side stream fork used; releases the
    // fork lock.  Returns false if a wait could not be enqueued.
    bool join(hipStream_t s)
    {
        bool ok = true;
        for (int k = 0; k < forked_; ++k)
            ok = ok && hipEventRecord(cur_->joined[k], cur_->side[k]) == hipSuccess &&
                 hipStreamWaitEvent(s, cur_->joined[k], 0) == hipSuccess;
        forked_ = 0;
        cur_ = nullptr;
        mu_.unlock();
        return ok;
    }

private:
    static constexpr int kMaxDevices = 64;
    struct Dev {
        bool ready = false;
        hipStream_t side[kSideStreams] = {};
        hipEvent_t joined[kSideStreams] = {};
        hipEvent_t start = nullptr;
    };
    std::mutex mu_;
    Dev dev_[kMaxDevices];
    Dev *cur_ = nullptr;
    int forked_ = 0;
};

// Writes the job lists of a call's launches (each list's jobs, then the
// table of their start units and the total, each 256-byte aligned, list
// after list) into the head of the caller's workspace, in stream order and
// without waiting for the stream: all of them in one asynchronous copy from
// the pinned staging ring, or, while the stream is being captured into a
// graph (a replay would copy whatever the staging buffer then holds), by
// kernels that carry the jobs in their arguments.  An empty list gets no
// table (its JobList is left as it is).
hc_status upload_job_lists(std::vector<Job> *lists, const uint64_t *totals, int nlists, void *ws, hipStream_t s,
                           JobList *jl)
{
    char *base = static_cast<char *>(ws);
    std::vector<uint64_t> at(nlists), starts_at(nlists);
    uint64_t end = 0, used = 0;
    for (int c = 0; c < nlists; ++c) {
        if (lists[c].empty()) continue;
        const uint64_t count = lists[c].size();
        at[c] = end;
        starts_at[c] = at[c] + align256(count * sizeof(Job));
        used = starts_at[c] + 8 * (count + 1);
        end = starts_at[c] + align256(8 * (count + 1));
    }
    if (used == 0) return HC_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return HC_ERR_HIP;
    if (cs != hipStreamCaptureStatusNone) {
        for (int c = 0; c < nlists; ++c) {
            if (lists[c].empty()) continue;
            if (launch_put_jobs(lists[c].data(), (uint32_t)lists[c].size(), totals[c],
                                reinterpret_cast<Job *>(base + at[c]), reinterpret_cast<uint64_t *>(base + starts_at[c]),
                                s) != hipSuccess)
                return HC_ERR_HIP;
        }
    } else {
        const hipError_t e = JobStaging::get().copy(ws, used, s, [&](char *h) {
            for (int c = 0; c < nlists; ++c) {
                if (lists[c].empty()) continue;
                const size_t count = lists[c].size();
                memcpy(h + at[c], lists[c].data(), count * sizeof(Job));
                uint64_t *st = reinterpret_cast<uint64_t *>(h + starts_at[c]);
                for (size_t k = 0; k < count; ++k) st[k] = lists[c][k].unit_begin;
                st[count] = totals[c];
            }
        });
        if (e != hipSuccess) return HC_ERR_HIP;
    }
    for (int c = 0; c < nlists; ++c) {
        if (lists[c].empty()) continue;
        jl[c].jobs = reinterpret_cast<const Job *>(base + at[c]);
        jl[c].starts = reinterpret_cast<const uint64_t *>(base + starts_at[c]);
        jl[c].count = (uint32_t)lists[c].size();
        jl[c].one = empty_job();
    }
    return HC_OK;
}

hc_status upload_jobs(std::vector<Job> &jobs, uint64_t total_units, void *ws, hipStream_t s, JobList *jl)
{
    return upload_job_lists(&jobs, &total_units, 1, ws, s, jl);
}

}  // namespace

extern "C" hc_status hc_histogram(const uint8_t *d_in, uint64_t n, uint64_t *d_hist, void *stream)
{
    if (!d_hist || !aligned(d_hist, 8)) return HC_ERR_INVALID_ARG;
    if (n > 0 && (!d_in || !aligned(d_in, 16))) return HC_ERR_INVALID_ARG;
    Job j = empty_job();
    j.in = d_in;
    j.n = n;
    j.hist = d_hist;
    const uint64_t chunk = hist_chunk(n);
    const uint64_t units = (n + chunk - 1) / chunk;
    if (units > 0x7FFFFFFFull) return HC_ERR_INVALID_ARG;
    return hip_status(launch_histogram(single(j), units, chunk, static_cast<hipStream_t>(stream)));
}

extern "C" hc_status hc_encode_blocks(const uint8_t *d_in, uint64_t n, uint32_t block_size, hc_cb_handle cb,
                                      uint8_t *d_out, uint64_t out_cap, uint64_t *d_block_off,
                                      uint32_t *d_sub_idx, uint32_t sub_block, void *d_ws,
                                      uint64_t ws_bytes, uint32_t *d_err, void *stream)
{
    return hc::encode_blocks_ws(d_in, n, block_size, cb, d_out, out_cap, d_block_off, d_sub_idx, sub_block, d_ws,
                                ws_bytes, d_err, stream);
}

hc_status hc::encode_blocks_ws(const uint8_t *d_in, uint64_t n, uint32_t block_size, hc_cb_handle cb, uint8_t *d_out,
                               uint64_t out_cap, uint64_t *d_block_off, uint32_t *d_sub_idx, uint32_t sub_block,
                               void *d_ws, uint64_t ws_bytes, uint32_t *d_err, void *stream)
{
    if (!valid_block_size(block_size) || !valid_sub_block(sub_block)) return HC_ERR_INVALID_ARG;
    hc_status st = check_encode(d_in, n, block_size, cb, d_out, out_cap, d_block_off, d_sub_idx, sub_block);
    if (st != HC_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n == 0) return hip_status(launch_encode_empty(d_block_off, s));
    const uint64_t nb = num_blocks(n, block_size);
    const uint32_t qpt = tuned_qpt(block_size, cb->host.max_len);
    const uint64_t tiles = nb * tiles_per_block(block_size, qpt);
    if (!d_ws || !aligned(d_ws, 8)) return HC_ERR_INVALID_ARG;
    if (ws_bytes < encode_scratch_bytes(tiles, qpt)) return HC_ERR_NO_SPACE;
    if (tiles > 0x7FFFFFFFull) return HC_ERR_INVALID_ARG;  // grid limit
    Job j = empty_job();
    j.in = d_in;
    j.n = n;
    j.tb = cb->d_tables;
    j.out = d_out;
    j.block_off = d_block_off;
    j.sub_idx = d_sub_idx;
    return hip_status(launch_encode(single(j), tiles, block_size, qpt, cb->host.max_len, sub_block,
                                    d_ws, d_err, s, kStepAll, complete8(cb->host)));
}

extern "C" hc_status hc_walk_blocks(const uint8_t *d_in, uint64_t in_bytes, uint64_t nb, uint64_t *d_block_off,
                                    uint32_t *d_err, void *stream)
{
    if (!d_block_off || !aligned(d_block_off, 8)) return HC_ERR_INVALID_ARG;
    if (in_bytes > 0 && (!d_in || !aligned(d_in, 4) || (in_bytes & 3))) return HC_ERR_INVALID_ARG;
    return hip_status(launch_walk(d_in, in_bytes, nb, d_block_off, d_err, static_cast<hipStream_t>(stream)));
}

extern "C" hc_status hc_decode_blocks(const uint8_t *d_in, uint64_t in_bytes, uint64_t n, uint32_t block_size,
                                      hc_cb_handle cb, const uint64_t *d_block_off, const uint32_t *d_sub_idx,
                                      uint32_t sub_block, uint8_t *d_out, uint32_t *d_err, void *stream)
{
    if (!valid_block_size(block_size) || !valid_sub_block(sub_block)) return HC_ERR_INVALID_ARG;
    hc_status st = check_decode(d_in, in_bytes, n, cb, d_block_off, d_sub_idx, sub_block, d_out);
    if (st != HC_OK || n == 0) return st;
    const uint64_t groups = decode_groups(n, block_size, sub_block, d_sub_idx != nullptr, complete8(cb->host));
    if (groups > 0x7FFFFFFFull) return HC_ERR_INVALID_ARG;
    Job j = empty_job();
    j.in = d_in;
    j.in_bytes = in_bytes;
    j.n = n;
    j.tb = cb->d_tables;
    j.out = d_out;
    j.block_off = const_cast<uint64_t *>(d_block_off);
    j.sub_idx = const_cast<uint32_t *>(d_sub_idx);
    return hip_status(launch_decode(single(j), groups, block_size, cb->host.max_len, sub_block, d_sub_idx != nullptr,
                                    d_err, static_cast<hipStream_t>(stream), complete8(cb->host)));
}

extern "C" hc_status hc_decode_blocks_selfsync(const uint8_t *d_in, uint64_t in_bytes, uint64_t n,
                                               uint32_t block_size, hc_cb_handle cb, const uint64_t *d_block_off,
                                               uint8_t *d_out, uint32_t *d_err, void *stream)
{
    if (!valid_block_size(block_size)) return HC_ERR_INVALID_ARG;
    hc_status st = check_decode(d_in, in_bytes, n, cb, d_block_off, nullptr, 0, d_out);
    if (st != HC_OK || n == 0) return st;
    const uint64_t nb = num_blocks(n, block_size);
    if (nb > 0x7FFFFFFFull) return HC_ERR_INVALID_ARG;
    Job j = empty_job();
    j.in = d_in;
    j.in_bytes = in_bytes;
    j.n = n;
    j.tb = cb->d_tables;
    j.out = d_out;
    j.block_off = const_cast<uint64_t *>(d_block_off);
    return hip_status(launch_decode_sync(single(j), nb, block_size, cb->host.max_len, d_err,
                                         static_cast<hipStream_t>(stream)));
}

// ---------------------------------------------------------------------- batches
extern "C" uint64_t hc_batch_workspace_bytes(const hc_item *items, uint32_t count, uint32_t block_size)
{
    if (!items || block_size == 0) return 0;
    uint64_t nb = 0;
    for (uint32_t k = 0; k < count; ++k) nb += num_blocks(items[k].n, block_size);
    // + the 256-byte alignment of each encode class's stretch of scratch
    return job_table_bytes(count) + encode_scratch_bound(nb, block_size) + 256 * 4;
}

extern "C" hc_status hc_histogram_batch(const hc_item *items, uint32_t count, void *d_ws, uint64_t ws_bytes,
                                        void *stream)
{
    if (!items || count == 0 || !d_ws || !aligned(d_ws, 256)) return HC_ERR_INVALID_ARG;
    if (ws_bytes < job_table_bytes(count)) return HC_ERR_NO_SPACE;
    uint64_t total = 0;
    for (uint32_t k = 0; k < count; ++k) {
        const hc_item &it = items[k];
        if (!it.hist || !aligned(it.hist, 8)) return HC_ERR_INVALID_ARG;
        if (it.n > 0 && (!it.in || !aligned(it.in, 16))) return HC_ERR_INVALID_ARG;
        total += it.n;
    }
    const uint64_t chunk = hist_chunk(total);
    std::vector<Job> jobs(count);
    uint64_t units = 0;
    for (uint32_t k = 0; k < count; ++k) {
        Job j = empty_job();
        j.in = items[k].in;
        j.n = items[k].n;
        j.hist = items[k].hist;
        j.unit_begin = units;
        units += (items[k].n + chunk - 1) / chunk;
        jobs[k] = j;
    }
    if (units > 0x7FFFFFFFull) return HC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    JobList jl;
    hc_status st = upload_jobs(jobs, units, d_ws, s, &jl);
    if (st != HC_OK) return st;
    return hip_status(launch_histogram(jl, units, chunk, s));
}

namespace {

// The three encode steps over a batch; 'steps' selects which run (bit 0:
// lengths, bit 1: offsets, bit 2: packing).  Every step re-derives the same
// job table from the items, so the steps may be issued as separate calls on
// one stream, with the same workspace.
// Encode launch classes: complete 8-bit codes (copied, no length pass),
// then by longest code: the kernels' variants (codes joined two or one at a
// time between flushes, the tile shape, 64-bit codes) change at these
// lengths, and a launch takes the variant of its longest code, so each class
// gets launches of its own.  Other codes of <= 8 bits share the class of
// <= 16: joining four codes instead of two gains less than the extra
// launches' tails cost.
int encode_class(uint32_t max_len, bool c8)
{
    return c8 ? 0 : max_len <= 16 ? 1 : max_len <= (uint32_t)kPackedMaxLen ? 2 : 3;
}
constexpr int kEncodeClasses = 4;

hc_status encode_batch_steps(const hc_item *items, uint32_t count, uint32_t block_size, uint32_t sub_block,
                             void *d_ws, uint64_t ws_bytes, uint32_t *d_err, void *stream, uint32_t steps)
{
    if (!items || count == 0 || !d_ws || !aligned(d_ws, 256)) return HC_ERR_INVALID_ARG;
    if (!valid_block_size(block_size) || !valid_sub_block(sub_block)) return HC_ERR_INVALID_ARG;
    std::vector<Job> jobs[kEncodeClasses];
    uint32_t max_len[kEncodeClasses] = {8, 1, 1, 1};
    for (uint32_t k = 0; k < count; ++k) {
        const hc_item &it = items[k];
        hc_status st = check_encode(it.in, it.n, block_size, it.cb, it.out, it.out_cap, it.block_off, it.sub_idx,
                                    sub_block);
        if (st != HC_OK) return st;
    }
    for (uint32_t k = 0; k < count; ++k) {
        const hc_item &it = items[k];
        const uint32_t L = it.n > 0 ? it.cb->host.max_len : 1u;
        const int c = encode_class(L, it.n > 0 && complete8(it.cb->host));
        max_len[c] = L > max_len[c] ? L : max_len[c];
        Job j = empty_job();
        j.in = it.in;
        j.n = it.n;
        j.tb = it.cb->d_tables;
        j.out = it.out;
        j.block_off = it.block_off;
        j.sub_idx = it.sub_idx;
        jobs[c].push_back(j);
    }
    // per class: its tile shape (from its longest code), its tiles numbered
    // job after job, its job table, and its own stretch of the scratch
    uint32_t qpt[kEncodeClasses];
    uint64_t tiles[kEncodeClasses], scratch_at[kEncodeClasses + 1];
    const uint64_t head = job_table_bytes(count);
    scratch_at[0] = 0;
    for (int c = 0; c < kEncodeClasses; ++c) {
        qpt[c] = tuned_qpt(block_size, max_len[c]);
        const uint32_t tpb = tiles_per_block(block_size, qpt[c]);
        tiles[c] = 0;
        for (Job &j : jobs[c]) {
            j.unit_begin = tiles[c];
            tiles[c] += num_blocks(j.n, block_size) * tpb;
        }
        if (tiles[c] > 0x7FFFFFFFull) return HC_ERR_INVALID_ARG;
        scratch_at[c + 1] = scratch_at[c] + ((encode_scratch_bytes(tiles[c], qpt[c]) + 255) & ~uint64_t(255));
    }
    if (ws_bytes < head + scratch_at[kEncodeClasses]) return HC_ERR_NO_SPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (steps & kStepOffsets)
        for (uint32_t k = 0; k < count; ++k)
            if (items[k].n == 0 && launch_encode_empty(items[k].block_off, s) != hipSuccess) return HC_ERR_HIP;
    for (int c = 0; c < kEncodeClasses; ++c)
        if (tiles[c] == 0) jobs[c].clear();  // nothing to launch (only empty items)
    JobList jl[kEncodeClasses];
    hc_status st = upload_job_lists(jobs, tiles, kEncodeClasses, d_ws, s, jl);
    if (st != HC_OK) return st;
    int classes = 0;
    for (int c = 0; c < kEncodeClasses; ++c) classes += jobs[c].empty() ? 0 : 1;
    hipStream_t on[kEncodeClasses];
    SideStreams &side = SideStreams::get();
    side.fork(s, classes, on);
    // the copy class (0) last: the other classes' launches are resident
    // first and the copy's groups fill what they leave of each CU
    int used = 0;
    hipError_t e = hipSuccess;
    for (int c = kEncodeClasses - 1; c >= 0 && e == hipSuccess; --c) {
        if (jobs[c].empty()) continue;
        void *scratch = static_cast<char *>(d_ws) + head + scratch_at[c];
        e = launch_encode(jl[c], tiles[c], block_size, qpt[c], max_len[c], sub_block, scratch, d_err, on[used++],
                          steps, c == 0);
    }
    const bool joined = side.join(s);
    return e == hipSuccess && joined ? HC_OK : HC_ERR_HIP;
}

}  // namespace

extern "C" hc_status hc_encode_batch(const hc_item *items, uint32_t count, uint32_t block_size, uint32_t sub_block,
                                     void *d_ws, uint64_t ws_bytes, uint32_t *d_err, void *stream)
{
    return encode_batch_steps(items, count, block_size, sub_block, d_ws, ws_bytes, d_err, stream, kStepAll);
}

extern "C" hc_status hc_encode_lengths_batch(const hc_item *items, uint32_t count, uint32_t block_size,
                                             uint32_t sub_block, void *d_ws, uint64_t ws_bytes, uint32_t *d_err,
                                             void *stream)
{
    return encode_batch_steps(items, count, block_size, sub_block, d_ws, ws_bytes, d_err, stream, kStepLengths);
}

extern "C" hc_status hc_encode_offsets_batch(const hc_item *items, uint32_t count, uint32_t block_size,
                                             uint32_t sub_block, void *d_ws, uint64_t ws_bytes, uint32_t *d_err,
                                             void *stream)
{
    return encode_batch_steps(items, count, block_size, sub_block, d_ws, ws_bytes, d_err, stream, kStepOffsets);
}

extern "C" hc_status hc_encode_pack_batch(const hc_item *items, uint32_t count, uint32_t block_size,
                                          uint32_t sub_block, void *d_ws, uint64_t ws_bytes, uint32_t *d_err,
                                          void *stream)
{
    return encode_batch_steps(items, count, block_size, sub_block, d_ws, ws_bytes, d_err, stream, kStepPack);
}

// Decode launch classes: complete 8-bit codes (the copy form), then the
// table decoder's variants by longest code (<= 8, 10, 12, 16, 24 bits, and
// longer), each launch taking the variant of its longest code.
int decode_class(const hc_codebook &cb)
{
    if (complete8(cb)) return 0;
    const uint32_t L = cb.max_len;
    return L <= 8 ? 1 : L <= 10 ? 2 : L <= 12 ? 3 : L <= 16 ? 4 : L <= (uint32_t)kPackedMaxLen ? 5 : 6;
}
constexpr int kDecodeClasses = 7;

extern "C" hc_status hc_decode_batch(const hc_item *items, uint32_t count, uint32_t block_size, uint32_t sub_block,
                                     void *d_ws, uint64_t ws_bytes, uint32_t *d_err, void *stream)
{
    if (!items || count == 0 || !d_ws || !aligned(d_ws, 256)) return HC_ERR_INVALID_ARG;
    if (!valid_block_size(block_size) || !valid_sub_block(sub_block)) return HC_ERR_INVALID_ARG;
    if (ws_bytes < job_table_bytes(count)) return HC_ERR_NO_SPACE;
    std::vector<Job> jobs[kDecodeClasses];
    uint64_t groups[kDecodeClasses] = {0, 0, 0, 0, 0, 0, 0};
    uint32_t max_len[kDecodeClasses] = {8, 1, 1, 1, 1, 1, 1};
    for (uint32_t k = 0; k < count; ++k) {
        const hc_item &it = items[k];
        hc_status st = check_decode(it.in, it.in_bytes, it.n, it.cb, it.block_off, it.sub_idx, sub_block, it.out);
        if (st != HC_OK) return st;
        if (it.n == 0) continue;  // nothing to decode
        const int c = decode_class(it.cb->host);
        Job j = empty_job();
        j.in = it.in;
        j.in_bytes = it.in_bytes;
        j.n = it.n;
        j.tb = it.cb->d_tables;
        j.out = it.out;
        j.block_off = it.block_off;
        j.sub_idx = it.sub_idx;
        j.unit_begin = groups[c];
        groups[c] += decode_groups(it.n, block_size, sub_block, sub_block != 0, c == 0);
        if (it.cb->host.max_len > max_len[c]) max_len[c] = it.cb->host.max_len;
        jobs[c].push_back(j);
    }
    for (int c = 0; c < kDecodeClasses; ++c)
        if (groups[c] > 0x7FFFFFFFull) return HC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    JobList jl[kDecodeClasses];
    hc_status st = upload_job_lists(jobs, groups, kDecodeClasses, d_ws, s, jl);
    if (st != HC_OK) return st;
    int classes = 0;
    for (int c = 0; c < kDecodeClasses; ++c) classes += jobs[c].empty() ? 0 : 1;
    hipStream_t on[kDecodeClasses];
    SideStreams &side = SideStreams::get();
    side.fork(s, classes, on);
    // the copy class (0) last, as in the encode
    int used = 0;
    hipError_t e = hipSuccess;
    for (int c = kDecodeClasses - 1; c >= 0 && e == hipSuccess; --c) {
        if (jobs[c].empty()) continue;
        e = launch_decode(jl[c], groups[c], block_size, max_len[c], sub_block, sub_block != 0, d_err, on[used++],
                          c == 0);
    }
    const bool joined = side.join(s);
    return e == hipSuccess && joined ? HC_OK : HC_ERR_HIP;
}

extern "C" hc_status hc_decode_batch_selfsync(const hc_item *items, uint32_t count, uint32_t block_size, void *d_ws,
                                              uint64_t ws_bytes, uint32_t *d_err, void *stream)
{
    if (!items || count == 0 || !d_ws || !aligned(d_ws, 256)) return HC_ERR_INVALID_ARG;
    if (!valid_block_size(block_size)) return HC_ERR_INVALID_ARG;
    if (ws_bytes < job_table_bytes(count)) return HC_ERR_NO_SPACE;
    // the classes of hc_decode_batch: complete 8-bit codes by the copy form
    // (which needs no index), the others by the piece decoder, one launch per
    // class (its payload copy sized for the class's longest code)
    std::vector<Job> jobs[kDecodeClasses];
    uint64_t units[kDecodeClasses] = {0, 0, 0, 0, 0, 0, 0};
    uint32_t max_len[kDecodeClasses] = {8, 1, 1, 1, 1, 1, 1};
    for (uint32_t k = 0; k < count; ++k) {
        const hc_item &it = items[k];
        hc_status st = check_decode(it.in, it.in_bytes, it.n, it.cb, it.block_off, nullptr, 0, it.out);
        if (st != HC_OK) return st;
        if (it.n == 0) continue;  // nothing to decode
        const int c = decode_class(it.cb->host);
        Job j = empty_job();
        j.in = it.in;
        j.in_bytes = it.in_bytes;
        j.n = it.n;
        j.tb = it.cb->d_tables;
        j.out = it.out;
        j.block_off = it.block_off;
        j.unit_begin = units[c];
        units[c] += c == 0 ? decode_groups(it.n, block_size, 0, false, true) : num_blocks(it.n, block_size);
        if (it.cb->host.max_len > max_len[c]) max_len[c] = it.cb->host.max_len;
        jobs[c].push_back(j);
    }
    for (int c = 0; c < kDecodeClasses; ++c)
        if (units[c] > 0x7FFFFFFFull) return HC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    JobList jl[kDecodeClasses];
    hc_status st = upload_job_lists(jobs, units, kDecodeClasses, d_ws, s, jl);
    if (st != HC_OK) return st;
    int classes = 0;
    for (int c = 0; c < kDecodeClasses; ++c) classes += jobs[c].empty() ? 0 : 1;
    hipStream_t on[kDecodeClasses];
    SideStreams &side = SideStreams::get();
    side.fork(s, classes, on);
    int used = 0;
    hipError_t e = hipSuccess;
    for (int c = kDecodeClasses - 1; c >= 0 && e == hipSuccess; --c) {  // the copy class last
        if (jobs[c].empty()) continue;
        hipStream_t sc = on[used++];
        e = c == 0 ? launch_decode(jl[c], units[c], block_size, 8, 0, false, d_err, sc, true)
                   : launch_decode_sync(jl[c], units[c], block_size, max_len[c], d_err, sc);
    }
    const bool joined = side.join(s);
    return e == hipSuccess && joined ? HC_OK : HC_ERR_HIP;
}
