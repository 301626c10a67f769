// Batched ensemble: many independent lattices (replicas of uneven L, r and
// seed) advanced together.  Every launch covers one row residue of one sweep
// of every replica: the waves of the launch are dealt out replica by replica
// (each replica's waves padded to whole workgroups, so a workgroup serves one
// replica and shares its threshold table), and each wave runs the segment
// update of one row segment.  A chunk of sweeps -- zeroing the per-sweep
// counters, 4 launches per sweep, the per-replica count scan and the advance
// of every replica's sweep index -- is captured once in a hipGraph and
// replayed; the sweep index lives in device memory so the same graph serves
// every chunk.  Results are those of the replicas run one by one.  This file
// is the host engine; the kernels and their launchers are pgg_ens_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "pgg.h"
#include "pgg_internal.hpp"

// ---------------------------------------------------------------------------
// Host engine behind the pgg_ensemble_* calls.
// ---------------------------------------------------------------------------
#define eerr pgg::set_errorf

struct pgg_ensemble {
    hipStream_t stream = nullptr;
    bool own_stream = false;  // graphs cannot capture the null stream
    // Graphs are captured on a private non-blocking stream (a capture on a
    // blocking stream is invalidated by another thread's null-stream work)
    // and launched on `stream`.
    hipStream_t capture_stream = nullptr;
    // Concurrent replica groups: the replicas are cut into `branches`
    // contiguous ranges of about equal work (sum of L^2); each range's chunk
    // is its own chain of launches, and the chains run side by side as
    // parallel branches of the chunk's graph (so one range's launch tails
    // overlap the other ranges' launches).  Group g: replicas first[g] ..
    // first[g] + count[g] - 1, waves[g] waves per launch.
    int branches = 1;
    std::vector<int> grp_first, grp_count, grp_waves;
    std::vector<hipStream_t> branch_streams;
    std::vector<hipEvent_t> branch_events;  // fork event, then one join event per branch
    // Replicas swept by the resident kernel (a whole chunk per launch, one
    // workgroup of res_waves waves per replica, the lattice in LDS): their
    // indices, on the device, and the largest side among them.  They run as
    // one more parallel branch beside the segment launches.
    int n_res = 0, res_L_max = 0, res_waves = 8;
    int* d_res_idx = nullptr;
    int device = 0;
    int n = 0;
    int chunk = 32;          // sweeps per graph replay
    int wpg = pgg::kWavesPerGroup;  // waves (segments of one replica) per workgroup
    int total_waves = 0;     // the tiled schedule: workgroups of a launch
    bool tiled = false;      // every replica runs the double tiling of Sec. IV
    size_t lds = 0;
    std::vector<pgg::EnsRep> host_reps;
    pgg::EnsRep* d_reps = nullptr;
    uint32_t* d_lattices = nullptr;
    uint32_t* d_tables = nullptr;
    unsigned long long* d_delta = nullptr;   // n * chunk * kSweepWords
    unsigned long long* d_counts = nullptr;  // n * chunk
    unsigned long long* d_nc = nullptr;      // n
    std::map<int, hipGraphExec_t> graphs;    // by chunk length
    std::vector<hipGraph_t> graph_defs;
    uint64_t t = 0;
    bool poisoned = false;
};

namespace {

pgg_status efail(pgg_ensemble* e, hipError_t err, const char* what) {
    eerr("%s: %s", what, hipGetErrorString(err));
    if (e) e->poisoned = true;
    return PGG_E_DEVICE;
}

#define ENS_HIP(e, call)                                            \
    do {                                                            \
        hipError_t err_ = (call);                                   \
        if (err_ != hipSuccess) return efail((e), err_, #call);     \
    } while (0)

void ens_release(pgg_ensemble* e) {
    if (!e) return;
    (void)hipStreamSynchronize(e->stream);
    for (auto& kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipGraph_t g : e->graph_defs) (void)hipGraphDestroy(g);
    if (e->d_reps) (void)hipFree(e->d_reps);
    if (e->d_res_idx) (void)hipFree(e->d_res_idx);
    if (e->d_lattices) (void)hipFree(e->d_lattices);
    if (e->d_tables) (void)hipFree(e->d_tables);
    if (e->d_delta) (void)hipFree(e->d_delta);
    if (e->d_counts) (void)hipFree(e->d_counts);
    if (e->d_nc) (void)hipFree(e->d_nc);
    // events before the streams they were recorded on
    for (hipEvent_t ev : e->branch_events) (void)hipEventDestroy(ev);
    if (e->capture_stream) (void)hipStreamDestroy(e->capture_stream);
    for (hipStream_t bs : e->branch_streams) (void)hipStreamDestroy(bs);
    if (e->own_stream && e->stream) (void)hipStreamDestroy(e->stream);
    delete e;
}

hipError_t enqueue_chunk(pgg_ensemble* e, int len, hipStream_t st) {
    if (e->tiled)
        return pgg::launch_ens_tiled_chunk(e->d_reps, e->n, e->total_waves, len, e->chunk, e->d_counts, st);
    if (e->branches == 1 && e->n_res == 0)
        return pgg::launch_ens_chunk(e->d_reps, e->n, e->total_waves, e->lds, len, e->chunk, true, e->d_counts, st,
                                     e->wpg);
    // the chunk's bookkeeping for every replica, then a fork: every segment
    // group runs its residue launches on a stream of its own, the resident
    // replicas theirs on another, and st waits for them all (a graph with
    // parallel branches) before the counts are scanned
    hipError_t err = pgg::launch_ens_begin(e->d_reps, e->n, len, e->chunk, true, st);
    if (err == hipSuccess) err = hipEventRecord(e->branch_events[0], st);
    int b = 0;
    for (int g = 0; err == hipSuccess && g < e->branches; ++g) {
        if (e->grp_waves[g] == 0) continue;  // a range of resident replicas only
        hipStream_t bs = e->branch_streams[b];
        err = hipStreamWaitEvent(bs, e->branch_events[0], 0);
        for (int q = 0; err == hipSuccess && q < len; ++q)
            for (int a = 0; err == hipSuccess && a < 4; ++a)
                err = pgg::launch_ens_residue(e->d_reps + e->grp_first[g], e->grp_count[g], e->grp_waves[g], e->lds,
                                              a, q, bs, e->wpg);
        if (err == hipSuccess) err = hipEventRecord(e->branch_events[1 + b], bs);
        if (err == hipSuccess) err = hipStreamWaitEvent(st, e->branch_events[1 + b], 0);
        ++b;
    }
    if (err == hipSuccess && e->n_res > 0) {
        hipStream_t bs = e->branch_streams[b];
        err = hipStreamWaitEvent(bs, e->branch_events[0], 0);
        if (err == hipSuccess)
            err = pgg::launch_ens_resident(e->d_reps, e->d_res_idx, e->n_res, e->res_L_max, e->res_waves, bs);
        if (err == hipSuccess) err = hipEventRecord(e->branch_events[1 + b], bs);
        if (err == hipSuccess) err = hipStreamWaitEvent(st, e->branch_events[1 + b], 0);
    }
    if (err == hipSuccess) err = pgg::launch_ens_end(e->d_reps, e->n, e->chunk, e->d_counts, st);
    return err;
}

hipError_t graph_for(pgg_ensemble* e, int len, hipGraphExec_t* out) {
    auto it = e->graphs.find(len);
    if (it != e->graphs.end()) { *out = it->second; return hipSuccess; }
    hipGraph_t g = nullptr;
    hipError_t err = hipSuccess;
    if (!e->capture_stream) err = hipStreamCreateWithFlags(&e->capture_stream, hipStreamNonBlocking);
    if (err != hipSuccess) return err;
    err = hipStreamBeginCapture(e->capture_stream, hipStreamCaptureModeThreadLocal);
    if (err != hipSuccess) return err;
    hipError_t enq = enqueue_chunk(e, len, e->capture_stream);
    err = hipStreamEndCapture(e->capture_stream, &g);
    if (enq != hipSuccess) { if (g) (void)hipGraphDestroy(g); return enq; }
    if (err != hipSuccess) return err;
    hipGraphExec_t ex = nullptr;
    err = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (err != hipSuccess) { (void)hipGraphDestroy(g); return err; }
    e->graph_defs.push_back(g);
    e->graphs[len] = ex;
    err = hipGraphUpload(ex, e->stream);
    if (err != hipSuccess) return err;
    *out = ex;
    return hipSuccess;
}

// Parameter checks of pgg_ensemble_create (no device call).
pgg_status validate_reps(const pgg_params* reps, uint32_t n_reps, const uint32_t* tiles, uint32_t chunk) {
    if (!reps || n_reps == 0 || n_reps > 65536) { eerr("need 1..65536 replicas"); return PGG_E_INVAL; }
    if (chunk == 0 || chunk > 1024) { eerr("chunk must lie in [1, 1024]"); return PGG_E_INVAL; }
    for (uint32_t k = 0; k < n_reps; ++k) {
        const pgg_params& p = reps[k];
        if (p.L < 64 || p.L > 32768 || p.L % 4 != 0) { eerr("replica %u: L must be a multiple of 4 in [64, 32768]", k); return PGG_E_INVAL; }
        if (!std::isfinite(p.r) || p.r < 0.0) { eerr("replica %u: r must be finite and >= 0", k); return PGG_E_INVAL; }
        if (!std::isfinite(p.K) || !(p.K > 0.0)) { eerr("replica %u: K must be finite and > 0", k); return PGG_E_INVAL; }
        if (!(p.p0 >= 0.0 && p.p0 <= 1.0)) { eerr("replica %u: p0 must lie in [0, 1]", k); return PGG_E_INVAL; }
        if (p.layout != PGG_LAYOUT_BITS) { eerr("replica %u: ensembles use the bits layout", k); return PGG_E_INVAL; }
        if (p.kernel != PGG_KERNEL_AUTO && p.kernel != PGG_KERNEL_SEGMENT) { eerr("replica %u: ensembles use the segment kernel", k); return PGG_E_INVAL; }
        if (p.group != 0) { eerr("replica %u: group must be 0 (the ensemble's waves_per_group applies)", k); return PGG_E_INVAL; }
        if (p.game != PGG_GAME_PUBLIC_GOODS) { eerr("replica %u: ensembles run the public goods game", k); return PGG_E_INVAL; }
        if (p.schedule != PGG_SCHEDULE_COLOUR16 && p.schedule != PGG_SCHEDULE_TILED) { eerr("replica %u: unknown schedule", k); return PGG_E_INVAL; }
        if (p.schedule != reps[0].schedule) { eerr("replica %u: every replica of an ensemble runs the same schedule", k); return PGG_E_INVAL; }
        if (p.schedule == PGG_SCHEDULE_TILED && (p.L % 8 != 0 || (tiles && tiles[k] != 0))) {
            eerr("replica %u: the tiled schedule needs L %% 8 == 0 and tile 0", k);
            return PGG_E_INVAL;
        }
        const uint32_t w = tiles ? tiles[k] : 0;
        if (w != 0 && !pgg::segw_valid((int)p.L, (int)w)) { eerr("replica %u: tile must be a multiple of 32 and <= L - 32, or L (whole rows)", k); return PGG_E_INVAL; }
    }
    return PGG_OK;
}

}  // namespace

extern "C" {

pgg_status pgg_ensemble_create(const pgg_params* reps, uint32_t n_reps, const pgg_ensemble_tune* tune,
                               void* hip_stream, pgg_ensemble** out) {
    if (!out) { eerr("out is NULL"); return PGG_E_INVAL; }
    *out = nullptr;
    const uint32_t* tiles = tune ? tune->tiles : nullptr;
    const uint32_t chunk = tune ? tune->chunk : 32;
    const uint32_t branches = tune ? tune->branches : 0;
    const uint32_t res_max_L = tune ? tune->resident_max_L : 0;
    const pgg_status vs = validate_reps(reps, n_reps, tiles, chunk);
    if (vs != PGG_OK) return vs;
    const int wpg = (tune && tune->waves_per_group) ? (int)tune->waves_per_group : pgg::kWavesPerGroup;
    if (!pgg::ens_wpg_valid(wpg)) { eerr("waves_per_group must be 0, 2, 4 or 8"); return PGG_E_INVAL; }
    if (branches > 16) { eerr("branches must lie in [0, 16]"); return PGG_E_INVAL; }
    const bool tiled_sched = reps[0].schedule == PGG_SCHEDULE_TILED;
    if (branches > 1 && tiled_sched) { eerr("the tiled schedule runs one branch"); return PGG_E_INVAL; }
    if (res_max_L != 0 && (res_max_L < 64 || res_max_L > (uint32_t)pgg::kResidentMaxL || tiled_sched)) {
        eerr("resident_max_L must be 0, or in [64, %d] with the 16-colour schedule", pgg::kResidentMaxL);
        return PGG_E_INVAL;
    }
    const int res_waves = (tune && tune->resident_waves) ? (int)tune->resident_waves : 8;
    if (!pgg::resident_waves_valid(res_waves)) { eerr("resident_waves must be 0, 4, 8 or 16"); return PGG_E_INVAL; }
    pgg_ensemble* e = new (std::nothrow) pgg_ensemble();
    if (!e) { eerr("host allocation failed"); return PGG_E_NOMEM; }
    e->stream = (hipStream_t)hip_stream;
    if (!e->stream) {
        if (hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) != hipSuccess) { eerr("stream creation failed"); delete e; return PGG_E_DEVICE; }
        e->own_stream = true;
    }
    e->n = (int)n_reps;
    e->chunk = (int)chunk;
    e->wpg = wpg;
    e->res_waves = res_waves;
    e->tiled = tiled_sched;
    if (hipGetDevice(&e->device) != hipSuccess) { eerr("no HIP device"); ens_release(e); return PGG_E_DEVICE; }

    // Layout: lattices back to back (256-byte aligned), tables, per-replica waves.
    std::vector<size_t> lat_off(n_reps);
    std::vector<int> res_idx;
    size_t lat_words = 0;
    int max_words = 0;
    e->host_reps.resize(n_reps);
    int waves = 0;
    for (uint32_t k = 0; k < n_reps; ++k) {
        const pgg_params& p = reps[k];
        pgg::EnsRep& rp = e->host_reps[k];
        std::memset(&rp, 0, sizeof(rp));
        pgg::ens_geometry(rp, (int)p.L, tiles ? (int)tiles[k] : 0);
        rp.k0 = (uint32_t)p.seed;
        rp.k1 = (uint32_t)(p.seed >> 32);
        rp.t0 = 0;
        rp.wave_base = waves;
        rp.tiled = e->tiled ? 1 : 0;
        rp.resident = (res_max_L != 0 && p.L <= res_max_L && pgg::resident_fits((int)p.L)) ? 1 : 0;
        if (rp.resident) {
            res_idx.push_back((int)k);
            e->res_L_max = std::max(e->res_L_max, (int)p.L);
        }
        waves += e->tiled ? pgg::tiled_blocks(rp.L) : pgg::ens_waves(rp, wpg);
        lat_off[k] = lat_words;
        lat_words += (e->tiled ? 1 : 2) * (((size_t)rp.L * rp.stride + 63) & ~(size_t)63);  // lat (and lat2)
        if (!e->tiled && !rp.resident) max_words = std::max(max_words, pgg::ens_wave_words(rp));
    }
    e->n_res = (int)res_idx.size();
    e->total_waves = waves;
    e->lds = (e->tiled || max_words == 0) ? 0 : pgg::ens_lds_bytes(max_words, wpg);
    // contiguous replica ranges of about equal segment work (sum of L^2 over
    // the replicas that are not resident); wave_base restarts in each
    // unset: two groups for the 16-colour schedule (measured at least as
    // fast as one on every ensemble tried: +14 % on 256 replicas of L = 128
    // to 1024, +23 % on the 21-lattice L = 1024 r scan), one for the tiling
    const int want = branches ? (int)branches : (tiled_sched ? 1 : 2);
    e->branches = std::max(1, std::min<int>(want, (int)n_reps));
    {
        double total_work = 0.0;
        for (uint32_t k = 0; k < n_reps; ++k)
            if (!e->host_reps[k].resident) total_work += (double)reps[k].L * (double)reps[k].L;
        double acc = 0.0;
        int g = 0, base = 0;
        e->grp_first.assign(1, 0);
        for (uint32_t k = 0; k < n_reps; ++k) {
            pgg::EnsRep& rp = e->host_reps[k];
            // start the next range once this one holds its share of the work
            // (every range keeps at least one replica)
            if (g + 1 < e->branches && k > (uint32_t)e->grp_first[g] && !rp.resident &&
                acc >= total_work * (double)(g + 1) / (double)e->branches) {
                e->grp_waves.push_back(base);
                e->grp_count.push_back((int)k - e->grp_first[g]);
                e->grp_first.push_back((int)k);
                ++g;
                base = 0;
            }
            rp.wave_base = base;
            if (!e->tiled) base += pgg::ens_waves(rp, wpg);
            if (!rp.resident) acc += (double)reps[k].L * (double)reps[k].L;
        }
        e->grp_waves.push_back(base);
        e->grp_count.push_back((int)n_reps - e->grp_first[g]);
        e->branches = g + 1;
        if (e->tiled) {  // the tiled schedule keeps its one range and its own wave bases
            e->grp_first.assign(1, 0);
            e->grp_count.assign(1, (int)n_reps);
            e->grp_waves.assign(1, waves);
            int wb = 0;
            for (uint32_t k = 0; k < n_reps; ++k) {
                e->host_reps[k].wave_base = wb;
                wb += pgg::tiled_blocks(e->host_reps[k].L);
            }
        }
    }
    // one stream per segment range with waves, one for the resident replicas,
    // and a fork event plus one join event per stream (none when nothing forks)
    int n_streams = 0;
    for (int g = 0; g < e->branches; ++g) n_streams += e->grp_waves[g] > 0 ? 1 : 0;
    n_streams += e->n_res > 0 ? 1 : 0;
    const bool forks = !e->tiled && (e->branches > 1 || e->n_res > 0);
    for (int g = 0; forks && g < n_streams; ++g) {
        hipStream_t bs = nullptr;
        if (hipStreamCreateWithFlags(&bs, hipStreamNonBlocking) != hipSuccess) { eerr("stream creation failed"); ens_release(e); return PGG_E_DEVICE; }
        e->branch_streams.push_back(bs);
    }
    for (int g = 0; forks && g <= n_streams; ++g) {
        hipEvent_t ev = nullptr;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) { eerr("event creation failed"); ens_release(e); return PGG_E_DEVICE; }
        e->branch_events.push_back(ev);
    }
    if (e->n_res > 0 && pgg::resident_lds_bytes(e->res_L_max, e->res_waves) > pgg::max_dynamic_lds()) {
        eerr("resident replicas of side %d do not fit the LDS with %d waves", e->res_L_max, e->res_waves);
        ens_release(e);
        return PGG_E_INVAL;
    }
    if (e->lds > pgg::max_dynamic_lds()) {
        eerr("the widest replica layout (%d LDS words per wave) does not fit %d waves per workgroup", max_words, wpg);
        ens_release(e);
        return PGG_E_INVAL;
    }

    auto alloc = [&](void** ptr, size_t bytes) -> pgg_status {
        hipError_t err = hipMalloc(ptr, bytes);
        if (err != hipSuccess) {
            eerr("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(err));
            return err == hipErrorOutOfMemory ? PGG_E_NOMEM : PGG_E_DEVICE;
        }
        return PGG_OK;
    };
    pgg_status st = alloc((void**)&e->d_lattices, lat_words * sizeof(uint32_t));
    if (st == PGG_OK) st = alloc((void**)&e->d_tables, (size_t)n_reps * 160 * sizeof(uint32_t));
    if (st == PGG_OK) st = alloc((void**)&e->d_delta, (size_t)n_reps * chunk * pgg::kSweepWords * sizeof(unsigned long long));
    if (st == PGG_OK) st = alloc((void**)&e->d_counts, (size_t)n_reps * chunk * sizeof(unsigned long long));
    if (st == PGG_OK) st = alloc((void**)&e->d_nc, (size_t)n_reps * sizeof(unsigned long long));
    if (st == PGG_OK) st = alloc((void**)&e->d_reps, (size_t)n_reps * sizeof(pgg::EnsRep));
    if (st == PGG_OK && e->n_res > 0) st = alloc((void**)&e->d_res_idx, (size_t)e->n_res * sizeof(int));
    if (st != PGG_OK) { ens_release(e); return st; }
    for (uint32_t k = 0; k < n_reps; ++k) {
        pgg::EnsRep& rp = e->host_reps[k];
        rp.lat = e->d_lattices + lat_off[k];
        rp.lat2 = e->tiled ? nullptr : rp.lat + (((size_t)rp.L * rp.stride + 63) & ~(size_t)63);
        rp.T = e->d_tables + (size_t)k * 160;
        rp.delta = e->d_delta + (size_t)k * chunk * pgg::kSweepWords;
        rp.nc = e->d_nc + k;
    }
    // Fermi tables built on the host, 160 words apart like the device tables
    std::vector<uint32_t> tables((size_t)n_reps * 160, 0u);
    for (uint32_t k = 0; k < n_reps; ++k) pgg::fermi_table(reps[k].r, reps[k].K, tables.data() + (size_t)k * 160);
    hipError_t err = hipMemcpyAsync(e->d_reps, e->host_reps.data(), n_reps * sizeof(pgg::EnsRep),
                                    hipMemcpyHostToDevice, e->stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(e->d_tables, tables.data(), tables.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                             e->stream);
    if (err == hipSuccess && e->n_res > 0)
        err = hipMemcpyAsync(e->d_res_idx, res_idx.data(), res_idx.size() * sizeof(int), hipMemcpyHostToDevice,
                             e->stream);
    if (err == hipSuccess) err = pgg::launch_fill_u64(e->d_nc, n_reps, 0ull, e->stream);
    for (uint32_t k = 0; k < n_reps && err == hipSuccess; ++k) {
        const pgg::EnsRep& rp = e->host_reps[k];
        err = pgg::launch_init(PGG_LAYOUT_BITS, rp.lat, rp.L, rp.stride, reps[k].p0, reps[k].seed, e->d_nc + k, e->stream);
    }
    if (err == hipSuccess) err = hipStreamSynchronize(e->stream);  // also keeps `tables` alive until the copy
    if (err != hipSuccess) {
        eerr("ensemble initialisation failed: %s", hipGetErrorString(err));
        ens_release(e);
        return PGG_E_DEVICE;
    }
    *out = e;
    return PGG_OK;
}

pgg_status pgg_ensemble_sweep(pgg_ensemble* e, uint32_t n_sweeps, uint64_t* counts) {
    if (!e) { eerr("ensemble is NULL"); return PGG_E_INVAL; }
    if (e->poisoned) { eerr("ensemble poisoned by an earlier device error"); return PGG_E_STATE; }
    if (e->t + (uint64_t)n_sweeps > 4294967296ull) { eerr("sweep index would exceed 2^32"); return PGG_E_INVAL; }
    if (n_sweeps == 0) return PGG_OK;
    uint32_t done = 0;
    while (done < n_sweeps) {
        const int len = (int)std::min<uint32_t>((uint32_t)e->chunk, n_sweeps - done);
        hipGraphExec_t g = nullptr;
        ENS_HIP(e, graph_for(e, len, &g));
        ENS_HIP(e, hipGraphLaunch(g, e->stream));
        if (counts) {
            // counts is n_reps rows of n_sweeps; this chunk fills columns done .. done + len.
            ENS_HIP(e, hipMemcpy2DAsync(counts + done, (size_t)n_sweeps * sizeof(uint64_t), e->d_counts,
                                        (size_t)e->chunk * sizeof(unsigned long long), (size_t)len * sizeof(uint64_t),
                                        (size_t)e->n, hipMemcpyDeviceToHost, e->stream));
            ENS_HIP(e, hipStreamSynchronize(e->stream));
        }
        done += (uint32_t)len;
    }
    e->t += n_sweeps;
    return PGG_OK;
}

pgg_status pgg_ensemble_coop_counts(pgg_ensemble* e, uint64_t* n_c) {
    if (!e || !n_c) { eerr("NULL argument"); return PGG_E_INVAL; }
    if (e->poisoned) { eerr("ensemble poisoned by an earlier device error"); return PGG_E_STATE; }
    ENS_HIP(e, hipMemcpyAsync(n_c, e->d_nc, (size_t)e->n * sizeof(uint64_t), hipMemcpyDeviceToHost, e->stream));
    ENS_HIP(e, hipStreamSynchronize(e->stream));
    return PGG_OK;
}

pgg_status pgg_ensemble_sweep_index(const pgg_ensemble* e, uint64_t* t) {
    if (!e || !t) { eerr("NULL argument"); return PGG_E_INVAL; }
    *t = e->t;
    return PGG_OK;
}

pgg_status pgg_ensemble_read_lattice(pgg_ensemble* e, uint32_t rep, uint8_t* host_LxL) {
    if (!e || !host_LxL) { eerr("NULL argument"); return PGG_E_INVAL; }
    if (rep >= (uint32_t)e->n) { eerr("replica %u out of range", rep); return PGG_E_INVAL; }
    if (e->poisoned) { eerr("ensemble poisoned by an earlier device error"); return PGG_E_STATE; }
    const pgg::EnsRep& rp = e->host_reps[rep];
    const size_t n = (size_t)rp.L * rp.L;
    uint8_t* tmp = nullptr;
    hipError_t err = hipMalloc((void**)&tmp, n);
    if (err != hipSuccess) { eerr("staging allocation failed: %s", hipGetErrorString(err)); return PGG_E_NOMEM; }
    err = pgg::launch_unpack(rp.lat, tmp, rp.L, rp.stride, e->stream);
    if (err == hipSuccess) err = hipMemcpyAsync(host_LxL, tmp, n, hipMemcpyDeviceToHost, e->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
    (void)hipFree(tmp);
    if (err != hipSuccess) return efail(e, err, "ensemble read_lattice");
    return PGG_OK;
}

pgg_status pgg_ensemble_threshold_table(pgg_ensemble* e, uint32_t rep, uint32_t* host_T) {
    if (!e || !host_T) { eerr("NULL argument"); return PGG_E_INVAL; }
    if (rep >= (uint32_t)e->n) { eerr("replica %u out of range", rep); return PGG_E_INVAL; }
    if (e->poisoned) { eerr("ensemble poisoned by an earlier device error"); return PGG_E_STATE; }
    hipError_t err = hipMemcpyAsync(host_T, e->host_reps[rep].T, pgg::kTableSize * sizeof(uint32_t),
                                    hipMemcpyDeviceToHost, e->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
    if (err != hipSuccess) return efail(e, err, "ensemble threshold_table");
    return PGG_OK;
}

void pgg_ensemble_destroy(pgg_ensemble* e) { ens_release(e); }

pgg_status pgg_ensemble_autotune(const pgg_params* reps, uint32_t n_reps, uint32_t probe_sweeps, void* hip_stream,
                                 uint32_t* tiles_out, pgg_ensemble_tune* tune_out, double* ms_out) {
    if (!reps || !tiles_out || !tune_out) { eerr("NULL argument"); return PGG_E_INVAL; }
    if (probe_sweeps == 0 || probe_sweeps > 4096) { eerr("probe_sweeps must lie in [1, 4096]"); return PGG_E_INVAL; }
    const pgg_status vs = validate_reps(reps, n_reps, nullptr, 1);
    if (vs != PGG_OK) return vs;
    if (reps[0].schedule == PGG_SCHEDULE_TILED) { eerr("the tiled schedule has nothing to tune"); return PGG_E_INVAL; }
    std::vector<uint32_t> sizes;
    for (uint32_t k = 0; k < n_reps; ++k)
        if (std::find(sizes.begin(), sizes.end(), reps[k].L) == sizes.end()) sizes.push_back(reps[k].L);
    std::map<uint32_t, uint32_t> width;  // current choice per L (0 = automatic)
    for (uint32_t L : sizes) width[L] = 0;
    uint32_t chunk = 32, wpg = (uint32_t)pgg::kWavesPerGroup, branches = 1, res_max_L = 0, res_waves = 8;
    std::vector<uint64_t> nc(n_reps);
    std::vector<uint32_t> tiles(n_reps);
    // Every trial ensemble runs on one stream that outlives them all (the
    // caller's, or one made here), so the timing events are only ever
    // recorded on a live stream -- never re-recorded after the stream of an
    // earlier record has been destroyed.
    hipStream_t tune_stream = (hipStream_t)hip_stream;
    bool own_tune_stream = false;
    if (!tune_stream) {
        if (hipStreamCreateWithFlags(&tune_stream, hipStreamNonBlocking) != hipSuccess) {
            eerr("stream creation failed");
            return PGG_E_DEVICE;
        }
        own_tune_stream = true;
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess) {
        if (ev0) (void)hipEventDestroy(ev0);
        if (own_tune_stream) (void)hipStreamDestroy(tune_stream);
        eerr("event creation failed");
        return PGG_E_DEVICE;
    }
    // One trial: a fresh ensemble with the current choices, one untimed run
    // (graph capture, clocks) and the best of three timed runs of n_probe
    // sweeps each -- at least 64 and two replays of the chunk, so that the
    // graph replays, not their capture, are timed.  Trials of equal n_probe
    // must end with equal cooperator counts.
    std::map<uint32_t, std::vector<uint64_t>> fingerprints;  // by n_probe
    auto trial = [&](double* ms) -> pgg_status {
        const uint32_t n_probe = std::max(std::max(probe_sweeps, 64u), 2 * chunk);
        for (uint32_t k = 0; k < n_reps; ++k) tiles[k] = width[reps[k].L];
        pgg_ensemble* e = nullptr;
        const pgg_ensemble_tune tn = {tiles.data(), chunk, wpg, branches, res_max_L, res_waves};
        pgg_status st = pgg_ensemble_create(reps, n_reps, &tn, tune_stream, &e);
        if (st != PGG_OK) return st;
        st = pgg_ensemble_sweep(e, n_probe, nullptr);
        double best = 1e300;
        for (int rep = 0; rep < 3 && st == PGG_OK; ++rep) {
            hipError_t err = hipEventRecord(ev0, e->stream);
            if (err == hipSuccess) st = pgg_ensemble_sweep(e, n_probe, nullptr);
            if (err == hipSuccess && st == PGG_OK) err = hipEventRecord(ev1, e->stream);
            if (err == hipSuccess && st == PGG_OK) err = hipEventSynchronize(ev1);
            float f = 0.f;
            if (err == hipSuccess && st == PGG_OK) err = hipEventElapsedTime(&f, ev0, ev1);
            if (err != hipSuccess) { eerr("autotune timing: %s", hipGetErrorString(err)); st = PGG_E_DEVICE; }
            best = std::min(best, (double)f / n_probe);
        }
        if (st == PGG_OK) st = pgg_ensemble_coop_counts(e, nc.data());
        pgg_ensemble_destroy(e);
        if (st != PGG_OK) return st;
        std::vector<uint64_t>& fingerprint = fingerprints[n_probe];
        if (fingerprint.empty()) {
            fingerprint = nc;
        } else if (fingerprint != nc) {
            eerr("autotune: cooperator counts differ between tuning choices");
            return PGG_E_DEVICE;
        }
        *ms = best;
        return PGG_OK;
    };
    double best_ms = 0.0;
    pgg_status st = trial(&best_ms);  // warms the device; timed again below
    if (st == PGG_OK) st = trial(&best_ms);
    // widths: the distinct sides with the most work (sum of L^2) first, at
    // most kTunedSides of them; the others keep the automatic width
    std::map<uint32_t, double> work;
    for (uint32_t k = 0; k < n_reps; ++k) work[reps[k].L] += (double)reps[k].L * (double)reps[k].L;
    std::stable_sort(sizes.begin(), sizes.end(), [&](uint32_t a, uint32_t b) { return work[a] > work[b]; });
    constexpr size_t kTunedSides = 6;
    for (size_t q = 0; q < std::min(sizes.size(), kTunedSides) && st == PGG_OK; ++q) {
        const uint32_t L = sizes[q];
        const uint32_t cap = (L - 32) & ~31u;
        std::vector<uint32_t> cand;
        for (uint32_t w = 64; w < cap; w *= 2) cand.push_back(w);
        if (cap >= 32) cand.push_back(cap);
        cand.push_back(L);  // whole rows
        pgg::EnsRep geo;
        std::memset(&geo, 0, sizeof(geo));
        pgg::ens_geometry(geo, (int)L, 0);
        uint32_t best_w = width[L];
        for (uint32_t w : cand) {
            if (w == (uint32_t)geo.segw) continue;  // the automatic width, already timed
            width[L] = w;
            double ms = 0.0;
            st = trial(&ms);
            if (st != PGG_OK) break;
            if (ms < best_ms) { best_ms = ms; best_w = w; }
        }
        width[L] = best_w;
    }
    const uint32_t wpgs[] = {2, 4, 8};
    uint32_t best_wpg = wpg;
    for (uint32_t g : wpgs) {
        if (st != PGG_OK || g == best_wpg) continue;
        wpg = g;
        double ms = 0.0;
        st = trial(&ms);
        if (st == PGG_OK && ms < best_ms) { best_ms = ms; best_wpg = g; }
    }
    wpg = best_wpg;
    // concurrent groups and resident sweeps of the replicas that fit one
    // workgroup's LDS (a chunk per launch, beside the segment launches) are
    // tried together: the resident branch changes which group split is best
    bool any_res = false;
    uint32_t max_fit = 0;  // largest side that could run resident
    for (uint32_t k = 0; k < n_reps; ++k)
        if (pgg::resident_fits((int)reps[k].L)) {
            any_res = true;
            max_fit = std::max(max_fit, reps[k].L);
        }
    const uint32_t branch_counts[] = {1, 2, 4};
    // (resident sides up to 512 are accepted but not searched: on the
    // 256-replica workload the tuner's short probes favoured them while
    // 400-sweep runs were 5 % slower than without resident replicas)
    const uint32_t res_sides[] = {0, 128, 256};
    uint32_t best_branches = branches, best_res = res_max_L;
    for (uint32_t bcount : branch_counts) {
        for (uint32_t rl : res_sides) {
            if (st != PGG_OK || (bcount == best_branches && rl == best_res) || bcount > n_reps) continue;
            if (rl != 0 && (!any_res || (rl > 128 && max_fit <= rl / 2))) continue;  // same set as rl / 2
            branches = bcount;
            res_max_L = rl;
            double ms = 0.0;
            st = trial(&ms);
            if (st == PGG_OK && ms < best_ms) { best_ms = ms; best_branches = bcount; best_res = rl; }
        }
    }
    branches = best_branches;
    res_max_L = best_res;
    uint32_t best_res_waves = res_waves;
    const uint32_t res_wave_counts[] = {4, 16};
    for (uint32_t rw : res_wave_counts) {
        if (st != PGG_OK || res_max_L == 0) break;
        res_waves = rw;
        double ms = 0.0;
        st = trial(&ms);
        if (st == PGG_OK && ms < best_ms) { best_ms = ms; best_res_waves = rw; }
    }
    res_waves = best_res_waves;
    const uint32_t chunks[] = {8, 16, 32, 64, 128};
    uint32_t best_chunk = chunk;
    for (uint32_t c : chunks) {
        if (st != PGG_OK || c == best_chunk) continue;
        chunk = c;
        double ms = 0.0;
        st = trial(&ms);
        if (st == PGG_OK && ms < best_ms) { best_ms = ms; best_chunk = c; }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    if (own_tune_stream) {
        (void)hipStreamSynchronize(tune_stream);
        (void)hipStreamDestroy(tune_stream);
    }
    if (st != PGG_OK) return st;
    for (uint32_t k = 0; k < n_reps; ++k) {
        uint32_t w = width[reps[k].L];
        if (w == 0) {  // the automatic width, made explicit
            pgg::EnsRep rp;
            std::memset(&rp, 0, sizeof(rp));
            pgg::ens_geometry(rp, (int)reps[k].L, 0);
            w = (uint32_t)rp.segw;
        }
        tiles_out[k] = w;
    }
    tune_out->tiles = tiles_out;
    tune_out->chunk = best_chunk;
    tune_out->waves_per_group = best_wpg;
    tune_out->branches = best_branches;
    tune_out->resident_max_L = best_res;
    tune_out->resident_waves = best_res ? best_res_waves : 0;
    if (ms_out) *ms_out = best_ms;
    return PGG_OK;
}

pgg_status pgg_ensemble_run(const pgg_params* reps, uint32_t n_reps, uint32_t n_sweeps, uint64_t* counts,
                            const pgg_ensemble_tune* tune, void* hip_stream) {
    const pgg_status vs = validate_reps(reps, n_reps, tune ? tune->tiles : nullptr, tune ? tune->chunk : 1);
    if (vs != PGG_OK) return vs;
    std::vector<uint32_t> tiles;
    pgg_ensemble_tune tuned = {nullptr, 32, 0, 0, 0, 0};
    if (tune) {
        tuned = *tune;
    } else if (reps[0].schedule != PGG_SCHEDULE_TILED) {
        tiles.resize(n_reps);
        const pgg_status st = pgg_ensemble_autotune(reps, n_reps, 8, hip_stream, tiles.data(), &tuned, nullptr);
        if (st != PGG_OK) return st;
    }
    pgg_ensemble* e = nullptr;
    pgg_status st = pgg_ensemble_create(reps, n_reps, &tuned, hip_stream, &e);
    if (st != PGG_OK) return st;
    st = pgg_ensemble_sweep(e, n_sweeps, counts);
    if (st == PGG_OK) {
        const hipError_t err = hipStreamSynchronize(e->stream);
        if (err != hipSuccess) st = efail(e, err, "ensemble run");
    }
    pgg_ensemble_destroy(e);
    return st;
}

}  // extern "C"
