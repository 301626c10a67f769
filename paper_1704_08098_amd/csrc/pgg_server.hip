// Job server engine: continuous batching of simulation jobs on one GPU.
//
// Jobs (a parameter set and a number of sweeps) are submitted at any time
// and queue on the host.  Every step: (1) queued jobs are admitted in
// arrival order while their device footprint fits the HBM budget, then any
// later job that still fits is admitted too (backfill); an admitted job gets
// its lattice, threshold table and counters carved from one device arena and
// its initial state drawn on the device; (2) every resident job advances
// min(chunk, remaining) sweeps -- all of them in the same launches, each at
// its own sweep index, with the ensemble's segment kernels; (3) the counts
// of the chunk are copied out, and finished jobs are retired: their final
// lattice is copied out and their arena space is freed for the next
// admissions.  Lattices stay resident on the device for the whole life of a
// job.  A job's results are exactly those of pgg_init + pgg_sweep with the
// same parameters, whatever else runs beside it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "pgg.h"
#include "pgg_internal.hpp"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
public:
    explicit Arena(size_t size) : size_(size) { if (size) free_[0] = size; }
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
        used_ -= bytes;
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

private:
    size_t size_;
    std::map<size_t, size_t> free_;  // offset -> length
    size_t used_ = 0, peak_ = 0;
};

enum JobState { kQueued = 0, kRunning = 1, kDone = 2 };

struct Job {
    pgg_params p{};
    uint32_t n_sweeps = 0, done = 0;
    int state = kQueued;
    size_t off = 0, bytes = 0;  // arena placement
    pgg::EnsRep rep{};
    uint32_t table[pgg::kTableSize];  // host-built Fermi table, the source of the upload (stable map node)
    std::vector<uint64_t> counts;
    std::vector<uint8_t> lattice;
};

}  // namespace

struct pgg_server {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint32_t chunk = 16, max_resident = 0, max_L = 0;
    size_t budget = 0;
    char* d_arena = nullptr;
    Arena arena{0};
    pgg::EnsRep* d_reps = nullptr;
    unsigned long long* d_counts = nullptr;  // max_resident x chunk
    uint8_t* d_stage = nullptr;              // max_L^2 bytes for lattice read-out
    pgg::EnsRep* h_reps = nullptr;           // pinned staging of the replica table
    // A step's launches (a chunk of every resident job) are replayed from a
    // hipGraph captured once per (replica slots, waves) bucket: the replica
    // table is padded with idle replicas (n_active 0) up to the bucket's
    // slot count and the waves up to the bucket's wave count, so the same
    // graph serves every step with that bucket whatever jobs are resident.
    hipStream_t capture_stream = nullptr;
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_defs;
    uint32_t slots = 0;                      // d_reps / h_reps entries (max_resident rounded up)
    size_t lds = 0;                          // LDS of any job's waves (the largest over the sizes accepted)
    char* d_idle = nullptr;                  // buffers the idle replicas point at
    pgg::EnsRep idle{};
    std::vector<unsigned long long> h_counts;
    std::deque<uint64_t> queue;
    std::vector<uint64_t> resident;
    std::map<uint64_t, Job> jobs;
    std::vector<uint64_t> completed;         // since the last pgg_server_completed
    uint64_t next_id = 1;
    uint64_t updates_done = 0, jobs_done = 0;
    bool poisoned = false;
};

namespace {

#define serr pgg::set_errorf

pgg_status sfail(pgg_server* s, hipError_t e, const char* what) {
    serr("%s: %s", what, hipGetErrorString(e));
    if (s) s->poisoned = true;
    return PGG_E_DEVICE;
}

#define SRV_HIP(s, call)                                           \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return sfail((s), e_, #call);        \
    } while (0)

#define SRV_LIVE(s)                                                                 \
    do {                                                                            \
        if (!(s)) { serr("server is NULL"); return PGG_E_INVAL; }                  \
        if ((s)->poisoned) { serr("server poisoned by an earlier device error"); return PGG_E_STATE; } \
    } while (0)

size_t job_lattice_words(uint32_t L) { return (size_t)L * 2 * ((L + 63) / 64); }

// Device bytes of one job: lattice and its second buffer, threshold table,
// per-sweep counters of a chunk, N_C.
size_t job_footprint(uint32_t L, uint32_t chunk) {
    return 2 * align_up(job_lattice_words(L) * sizeof(uint32_t)) + align_up(160 * sizeof(uint32_t)) +
           align_up((size_t)chunk * pgg::kSweepWords * sizeof(unsigned long long)) +
           align_up(sizeof(unsigned long long));
}

bool job_params_ok(const pgg_params* p, uint32_t max_L, const char** why) {
    if (!p) { *why = "params is NULL"; return false; }
    if (p->L < 64 || p->L > max_L || p->L % 4 != 0) { *why = "L must be a multiple of 4 in [64, max_L]"; return false; }
    if (!std::isfinite(p->r) || p->r < 0.0) { *why = "r must be finite and >= 0"; return false; }
    if (!std::isfinite(p->K) || !(p->K > 0.0)) { *why = "K must be finite and > 0"; return false; }
    if (!(p->p0 >= 0.0 && p->p0 <= 1.0)) { *why = "p0 must lie in [0, 1]"; return false; }
    if (p->layout != PGG_LAYOUT_BITS) { *why = "jobs use the bits layout"; return false; }
    if (p->kernel != PGG_KERNEL_AUTO && p->kernel != PGG_KERNEL_SEGMENT) { *why = "jobs use the segment kernel"; return false; }
    if (p->tile != 0 && !pgg::segw_valid((int)p->L, (int)p->tile)) { *why = "tile must be a multiple of 32 and <= L - 32, or L for whole rows"; return false; }
    {
        pgg::EnsRep rp;
        std::memset(&rp, 0, sizeof(rp));
        pgg::ens_geometry(rp, (int)p->L, (int)p->tile);
        if (pgg::ens_lds_bytes(pgg::ens_wave_words(rp)) > pgg::max_dynamic_lds()) { *why = "tile too wide for the workgroup's LDS"; return false; }
    }
    if (p->group != 0) { *why = "jobs run with the server's workgroup shape (group must be 0)"; return false; }
    if (p->schedule != PGG_SCHEDULE_COLOUR16) { *why = "jobs run the 16-colour sweep"; return false; }
    if (p->game != PGG_GAME_PUBLIC_GOODS) { *why = "jobs run the public goods game"; return false; }
    return true;
}

// Place a queued job on the device and draw its initial state.
hipError_t admit(pgg_server* s, uint64_t id, Job& j) {
    j.state = kRunning;
    char* base = s->d_arena + j.off;
    pgg::EnsRep& rp = j.rep;
    std::memset(&rp, 0, sizeof(rp));
    pgg::ens_geometry(rp, (int)j.p.L, (int)j.p.tile);
    const size_t lat_b = align_up(job_lattice_words(j.p.L) * sizeof(uint32_t));
    const size_t tab_b = align_up(160 * sizeof(uint32_t));
    const size_t del_b = align_up((size_t)s->chunk * pgg::kSweepWords * sizeof(unsigned long long));
    rp.lat = (uint32_t*)base;
    rp.lat2 = (uint32_t*)(base + lat_b);
    rp.T = (const uint32_t*)(base + 2 * lat_b);
    rp.delta = (unsigned long long*)(base + 2 * lat_b + tab_b);
    rp.nc = (unsigned long long*)(base + 2 * lat_b + tab_b + del_b);
    rp.k0 = (uint32_t)j.p.seed;
    rp.k1 = (uint32_t)(j.p.seed >> 32);
    rp.t0 = 0;
    s->resident.push_back(id);
    pgg::fermi_table(j.p.r, j.p.K, j.table);
    hipError_t e = pgg::upload_table(j.table, (uint32_t*)rp.T, s->stream);
    if (e == hipSuccess) e = pgg::launch_init(PGG_LAYOUT_BITS, rp.lat, rp.L, rp.stride, j.p.p0, j.p.seed, rp.nc, s->stream);
    return e;
}

// Buckets: replica slots rounded up to a power of two (at least 8), waves up
// to a multiple of an eighth of their power of two (at least 64), so that the
// padding costs at most about an eighth of a launch in idle workgroups.
int slot_bucket(int n) {
    int b = 8;
    while (b < n) b <<= 1;
    return b;
}
int wave_bucket(int w) {
    int p = 64;
    while (p < w) p <<= 1;
    const int step = std::max(64, p / 8);
    return (w + step - 1) / step * step;
}

// The graph of one step for a bucket (captured on first use).
hipError_t step_graph(pgg_server* s, int slots, int waves, hipGraphExec_t* out) {
    const auto key = std::make_pair(slots, waves);
    auto it = s->graphs.find(key);
    if (it != s->graphs.end()) { *out = it->second; return hipSuccess; }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t enq = pgg::launch_ens_chunk(s->d_reps, slots, waves, s->lds, (int)s->chunk, (int)s->chunk, false,
                                                 s->d_counts, s->capture_stream);
    e = hipStreamEndCapture(s->capture_stream, &g);
    if (enq != hipSuccess) { if (g) (void)hipGraphDestroy(g); return enq; }
    if (e != hipSuccess) return e;
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return e; }
    s->graph_defs.push_back(g);
    s->graphs[key] = ex;
    *out = ex;
    return hipSuccess;
}

void server_release(pgg_server* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    if (s->d_arena) (void)hipFree(s->d_arena);
    if (s->d_reps) (void)hipFree(s->d_reps);
    if (s->d_counts) (void)hipFree(s->d_counts);
    if (s->d_stage) (void)hipFree(s->d_stage);
    if (s->h_reps) (void)hipHostFree(s->h_reps);
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipGraph_t g : s->graph_defs) (void)hipGraphDestroy(g);
    if (s->d_idle) (void)hipFree(s->d_idle);
    if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // namespace

extern "C" {

size_t pgg_server_job_bytes(uint32_t L, uint32_t chunk) { return job_footprint(L, chunk); }

pgg_status pgg_server_create(size_t hbm_budget, uint32_t max_L, uint32_t max_resident, uint32_t chunk,
                             void* hip_stream, pgg_server** out) {
    if (!out) { serr("out is NULL"); return PGG_E_INVAL; }
    *out = nullptr;
    if (chunk == 0 || chunk > 1024) { serr("chunk must lie in [1, 1024]"); return PGG_E_INVAL; }
    if (max_L < 64 || max_L > 32768 || max_L % 4 != 0) { serr("max_L must be a multiple of 4 in [64, 32768]"); return PGG_E_INVAL; }
    if (max_resident == 0 || max_resident > 65536) { serr("max_resident must lie in [1, 65536]"); return PGG_E_INVAL; }
    if (hbm_budget < job_footprint(64, chunk)) { serr("budget below the smallest job's footprint"); return PGG_E_INVAL; }
    pgg_server* s = new (std::nothrow) pgg_server();
    if (!s) { serr("host allocation failed"); return PGG_E_NOMEM; }
    s->chunk = chunk;
    s->max_L = max_L;
    s->max_resident = max_resident;
    s->budget = hbm_budget & ~(kAlign - 1);
    s->arena = Arena(s->budget);
    s->stream = (hipStream_t)hip_stream;
    hipError_t e = hipSuccess;
    if (!s->stream) {
        e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        s->own_stream = (e == hipSuccess);
    }
    s->slots = (uint32_t)slot_bucket((int)max_resident);
    // the widest wave layout over every side a job may have
    {
        int words = 0;
        for (uint32_t L = 64; L <= max_L; L += 4) {
            pgg::EnsRep rp;
            std::memset(&rp, 0, sizeof(rp));
            pgg::ens_geometry(rp, (int)L, 0);
            words = std::max(words, pgg::ens_wave_words(rp));
        }
        s->lds = pgg::ens_lds_bytes(words);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_arena, s->budget);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_reps, (size_t)s->slots * sizeof(pgg::EnsRep));
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_counts, (size_t)s->slots * chunk * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_stage, (size_t)max_L * max_L);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_reps, (size_t)s->slots * sizeof(pgg::EnsRep), 0);
    // idle replicas: an L = 64 geometry, no active sweeps, and small buffers
    // for the table, counters and N_C that the bookkeeping kernels touch
    const size_t idle_tab = align_up(160 * sizeof(uint32_t));
    const size_t idle_del = align_up((size_t)chunk * pgg::kSweepWords * sizeof(unsigned long long));
    const size_t idle_lat = align_up(job_lattice_words(64) * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_idle, idle_tab + idle_del + 2 * idle_lat + kAlign);
    if (e == hipSuccess) {
        std::memset(&s->idle, 0, sizeof(s->idle));
        pgg::ens_geometry(s->idle, 64, 0);
        s->idle.T = (const uint32_t*)s->d_idle;
        s->idle.delta = (unsigned long long*)(s->d_idle + idle_tab);
        s->idle.lat = (uint32_t*)(s->d_idle + idle_tab + idle_del);
        s->idle.lat2 = (uint32_t*)(s->d_idle + idle_tab + idle_del + idle_lat);
        s->idle.nc = (unsigned long long*)(s->d_idle + idle_tab + idle_del + 2 * idle_lat);
        s->idle.n_active = 0;
        e = hipMemsetAsync(s->d_idle, 0, idle_tab + idle_del + 2 * idle_lat + kAlign, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    }
    if (e != hipSuccess) {
        serr("server allocation failed: %s", hipGetErrorString(e));
        const bool oom = e == hipErrorOutOfMemory;
        server_release(s);
        return oom ? PGG_E_NOMEM : PGG_E_DEVICE;
    }
    s->h_counts.resize((size_t)s->slots * chunk);
    *out = s;
    return PGG_OK;
}

pgg_status pgg_server_submit(pgg_server* s, const pgg_params* p, uint32_t n_sweeps, uint64_t* job_id) {
    SRV_LIVE(s);
    if (!job_id) { serr("job_id is NULL"); return PGG_E_INVAL; }
    const char* why = nullptr;
    if (!job_params_ok(p, s->max_L, &why)) { serr("invalid job: %s", why); return PGG_E_INVAL; }
    if (n_sweeps == 0) { serr("a job needs at least one sweep"); return PGG_E_INVAL; }
    if (job_footprint(p->L, s->chunk) > s->budget) { serr("the job's footprint exceeds the whole budget"); return PGG_E_INVAL; }
    {
        // a step's launches reserve the LDS of the widest automatic layout
        pgg::EnsRep rp;
        std::memset(&rp, 0, sizeof(rp));
        pgg::ens_geometry(rp, (int)p->L, (int)p->tile);
        if (pgg::ens_lds_bytes(pgg::ens_wave_words(rp)) > s->lds) {
            serr("the job's tile needs more LDS per workgroup than the server's launches reserve (use tile 0)");
            return PGG_E_INVAL;
        }
    }
    const uint64_t id = s->next_id++;
    Job& j = s->jobs[id];
    j.p = *p;
    j.n_sweeps = n_sweeps;
    j.bytes = job_footprint(p->L, s->chunk);
    s->queue.push_back(id);
    *job_id = id;
    return PGG_OK;
}

pgg_status pgg_server_step(pgg_server* s, uint32_t* n_resident) {
    SRV_LIVE(s);
    // (1) admission: arrival order while the head fits, then backfill.
    bool head_blocked = false;
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        if (s->resident.size() >= s->max_resident) break;
        Job& j = s->jobs[*it];
        size_t off = 0;
        if (s->arena.alloc(j.bytes, &off)) {
            j.off = off;
            const uint64_t id = *it;
            it = s->queue.erase(it);
            SRV_HIP(s, admit(s, id, j));
        } else {
            head_blocked = true;  // later, smaller jobs may still fit (backfill)
            ++it;
        }
    }
    (void)head_blocked;
    const int n = (int)s->resident.size();
    if (n_resident) *n_resident = (uint32_t)n;
    if (n == 0) return PGG_OK;

    // (2) one chunk for every resident job, each at its own sweep index: the
    // replica table (padded with idle replicas to the bucket's slots) goes up,
    // and the bucket's graph runs chunk sweeps -- a job with fewer sweeps
    // left runs only its own n_active of them.
    int waves = 0;
    for (int k = 0; k < n; ++k) {
        Job& j = s->jobs[s->resident[k]];
        pgg::EnsRep rp = j.rep;
        rp.t0 = j.done;
        rp.n_active = (int)std::min<uint32_t>(s->chunk, j.n_sweeps - j.done);
        rp.wave_base = waves;
        waves += pgg::ens_waves(rp);
        s->h_reps[k] = rp;
    }
    const int slots = std::min<int>(slot_bucket(n), (int)s->slots);
    const int wave_pad = wave_bucket(waves);
    for (int k = n; k < slots; ++k) {
        s->h_reps[k] = s->idle;
        s->h_reps[k].wave_base = wave_pad;  // owns no wave of the launch
    }
    hipGraphExec_t g = nullptr;
    SRV_HIP(s, step_graph(s, slots, wave_pad, &g));
    SRV_HIP(s, hipMemcpyAsync(s->d_reps, s->h_reps, (size_t)slots * sizeof(pgg::EnsRep), hipMemcpyHostToDevice,
                              s->stream));
    SRV_HIP(s, hipGraphLaunch(g, s->stream));
    SRV_HIP(s, hipMemcpyAsync(s->h_counts.data(), s->d_counts, (size_t)n * s->chunk * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s->stream));
    SRV_HIP(s, hipStreamSynchronize(s->stream));

    // (3) collect counts, retire finished jobs: every finished lattice is
    // unpacked and copied out in stream order (the staging buffer is reused
    // in turn), with one synchronisation for all of them.
    std::vector<uint64_t> still, retired;
    still.reserve(n);
    for (int k = 0; k < n; ++k) {
        const uint64_t id = s->resident[k];
        Job& j = s->jobs[id];
        const uint32_t len = std::min<uint32_t>(s->chunk, j.n_sweeps - j.done);
        for (uint32_t q = 0; q < len; ++q) j.counts.push_back(s->h_counts[(size_t)k * s->chunk + q]);
        j.done += len;
        s->updates_done += (uint64_t)len * j.p.L * j.p.L;
        if (j.done < j.n_sweeps) { still.push_back(id); continue; }
        const size_t cells = (size_t)j.p.L * j.p.L;
        j.lattice.resize(cells);
        SRV_HIP(s, pgg::launch_unpack(j.rep.lat, s->d_stage, j.rep.L, j.rep.stride, s->stream));
        SRV_HIP(s, hipMemcpyAsync(j.lattice.data(), s->d_stage, cells, hipMemcpyDeviceToHost, s->stream));
        retired.push_back(id);
    }
    if (!retired.empty()) SRV_HIP(s, hipStreamSynchronize(s->stream));
    for (uint64_t id : retired) {
        Job& j = s->jobs[id];
        j.state = kDone;
        s->arena.release(j.off, j.bytes);
        s->completed.push_back(id);
        s->jobs_done += 1;
    }
    s->resident.swap(still);
    return PGG_OK;
}

pgg_status pgg_server_completed(pgg_server* s, uint64_t* ids, uint32_t cap, uint32_t* n) {
    SRV_LIVE(s);
    if (!n || (cap && !ids)) { serr("NULL argument"); return PGG_E_INVAL; }
    const uint32_t m = (uint32_t)std::min<size_t>(cap, s->completed.size());
    for (uint32_t k = 0; k < m; ++k) ids[k] = s->completed[k];
    s->completed.erase(s->completed.begin(), s->completed.begin() + m);
    *n = m;
    return PGG_OK;
}

pgg_status pgg_server_job_state(pgg_server* s, uint64_t id, int* state, uint32_t* sweeps_done) {
    SRV_LIVE(s);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) { serr("unknown job %llu", (unsigned long long)id); return PGG_E_INVAL; }
    if (state) *state = it->second.state;
    if (sweeps_done) *sweeps_done = it->second.done;
    return PGG_OK;
}

pgg_status pgg_server_job_result(pgg_server* s, uint64_t id, uint64_t* counts, uint8_t* lattice) {
    SRV_LIVE(s);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) { serr("unknown job %llu", (unsigned long long)id); return PGG_E_INVAL; }
    Job& j = it->second;
    if (j.state != kDone) { serr("job %llu has not finished", (unsigned long long)id); return PGG_E_INVAL; }
    if (counts) std::memcpy(counts, j.counts.data(), j.counts.size() * sizeof(uint64_t));
    if (lattice) std::memcpy(lattice, j.lattice.data(), j.lattice.size());
    s->jobs.erase(it);
    return PGG_OK;
}

pgg_status pgg_server_stats(const pgg_server* s, pgg_server_info* st) {
    if (!s || !st) { serr("NULL argument"); return PGG_E_INVAL; }
    st->queued = (uint32_t)s->queue.size();
    st->resident = (uint32_t)s->resident.size();
    st->completed = s->jobs_done;
    st->bytes_in_use = s->arena.used();
    st->peak_bytes = s->arena.peak();
    st->budget = s->budget;
    st->site_updates = s->updates_done;
    return PGG_OK;
}

void pgg_server_destroy(pgg_server* s) { server_release(s); }

}  // extern "C"
