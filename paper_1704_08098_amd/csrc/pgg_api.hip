// C ABI of the engine: validation, ownership, streams and error reporting
// around the kernels.  Declarations and the contract are in include/pgg.h.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "pgg.h"
#include "pgg_internal.hpp"

namespace {

thread_local char g_err[512] = "";

void set_err(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

constexpr uint32_t kChunk = 4096;  // sweeps per count-history chunk
constexpr int kGraphChunk = 64;    // sweeps per graph replay (segment kernel)
constexpr int kKernelTiled = 100;  // internal kernel id of the tiled schedule (not a pgg_kernel value)
constexpr int kKernelPd = 101;     // internal kernel id of the pairwise game (8-colour schedule)
// Largest L for which AUTO takes the resident kernel: a sweep costs it 16-17 us
// at L = 64 and 19-22 us at L = 128 against 31-35 us for the whole-row segment
// kernel's four launches; at L = 256 it is 30-45 us against 33-36 us,
// depending on how many sites are active.
constexpr uint32_t kResidentAutoMaxL = 128;

}  // namespace

namespace pgg {
void set_errorf(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

size_t max_dynamic_lds() {
    constexpr size_t kFallback = 64 * 1024;
    constexpr int kDevices = 64;
    static std::atomic<size_t> cache[kDevices];  // 0 = not looked up yet
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevices) return kFallback;
    size_t v = cache[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        int bytes = 0;
        v = (hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
             bytes >= (int)kFallback)
                ? (size_t)bytes
                : kFallback;
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

bool allow_dynamic_lds(const void* kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return true;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess) return true;
    (void)hipGetLastError();  // leave no sticky error behind
    return false;
}
}  // namespace pgg

struct pgg_sim {
    pgg_params p;
    hipStream_t stream = nullptr;
    int device = 0;
    void* lattice = nullptr;
    bool owns_lattice = false;
    uint32_t* lattice2 = nullptr;  // segment kernel: odd sweeps of a call land here
    uint32_t* shadow = nullptr;    // int8 layout on the segment, resident and tiled paths: bit-packed working lattice
    // Segment kernel: run as a one-replica ensemble.  d_rep[0] serves the
    // captured chunks (one graph per chunk length), d_rep[1] the eager
    // launches of timing mode (it also counts draws); sweep indices live in
    // device memory.
    pgg::EnsRep seg_rep;
    pgg::EnsRep* d_rep = nullptr;
    unsigned long long* d_gdelta = nullptr;   // kGraphChunk x kSweepWords
    unsigned long long* d_gcounts = nullptr;  // kGraphChunk
    hipStream_t capture_stream = nullptr;
    std::map<int, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_defs;
    int seg_waves = 0;
    size_t seg_lds = 0;
    bool pair = false;  // SEGMENT_PAIR: two residues per launch
    int launches_per_sweep = 4;
    int wpg = pgg::kWavesPerGroup;
    int stride = 0;  // bits layout: 32-bit words per row
    int kernel = PGG_KERNEL_COLOUR;
    int R = 1;       // rows per workgroup (row-band kernels)
    int segw = 0;    // columns per segment (segment kernel)
    uint32_t* d_table = nullptr;
    uint32_t h_table[pgg::kTableSize];  // host copy, the source of the upload
    unsigned long long* d_nc = nullptr;
    // Per-sweep counters and count history of the non-segment paths, sized
    // for the longest chunk of sweeps a call has needed so far (at most
    // kChunk sweeps of kSweepWords words); the segment paths use d_gdelta.
    unsigned long long* d_delta = nullptr;
    unsigned long long* d_counts = nullptr;
    uint32_t delta_sweeps = 0;
    uint64_t t = 0;
    bool poisoned = false;
    // Diagnostics (pgg_set_kernel_timing): a pair of HIP events around every
    // launch of the sweep kernel, folded into the totals when read.
    bool timing = false;
    std::vector<hipEvent_t> events;  // pool; 2 per launch
    size_t events_used = 0;
    uint64_t timed_launches = 0;
    double timed_ms = 0.0;
    unsigned long long* d_drawn = nullptr;
    unsigned long long* d_span = nullptr;  // segment kernel, timing mode: kGraphChunk x 4 launches x kSpanWords
    double wall_khz = 0.0;
    hipEvent_t chunk_ev[2] = {nullptr, nullptr};  // segment kernel, timing mode
    uint64_t span_launches = 0;
    double span_us = 0.0;
    // Persistent strip kernel plan.
    pgg::StripTask* d_tasks = nullptr;
    int n_tasks = 0;
    int strip_G = 1;
    size_t strip_lds = 0;
    uint64_t* d_ring = nullptr;
    size_t ring_words = 0;
    uint32_t* d_abort = nullptr;
    uint64_t wait_ticks = 0;
};

namespace {

// Rows per workgroup for the row-band kernels: enough colour sites per
// class to occupy the workgroup's 256 lanes.
int choose_R(uint32_t L) {
    const int q4 = (int)L / 4;
    int R = (256 + q4 - 1) / q4;
    if (R > q4) R = q4;
    if (R < 1) R = 1;
    return R;
}

// Columns per segment: about 8 waves per SIMD at large L, at least 128
// columns (the 18-column margins stay cheap), at most L - 32.
// LDS bytes of a segment-kernel workgroup for side L, width segw, wpg waves.
size_t segment_lds(uint32_t L, int segw, int wpg) {
    pgg::EnsRep rp;
    std::memset(&rp, 0, sizeof(rp));
    pgg::ens_geometry(rp, (int)L, segw);
    return pgg::ens_lds_bytes(pgg::ens_wave_words(rp), wpg);
}

// Work split of the segment kernel: the automatic one, with segments
// narrowed until the workgroup's LDS fits.
int choose_segw(uint32_t L, int wpg) {
    // a single lattice needs its waves: whole rows (several per wave for L a
    // multiple of 32, one periodic row otherwise) only up to L = 1024, else
    // segments of about 1376 columns
    int w = L <= 1024 ? (int)L : pgg::split_segw((int)L);
    if (w == (int)L && segment_lds(L, w, wpg) <= pgg::max_dynamic_lds()) return w;
    if (w == (int)L) w = ((int)L - 32) & ~31;
    while (w > 32 && segment_lds(L, w, wpg) > pgg::max_dynamic_lds()) w -= 32;
    return w;
}

// Paired kernel: segments of about 2048 columns (at L = 4096: 128 bands x 2
// segments = 256 workgroups, one per CU), at most L - 64.  Measured at L =
// 4096 over sweeps 5..24: 39.4 us per sweep against 43.2 with 1024 columns
// (512 workgroups, two per CU) and 44.0 with 1536 -- a wave's class lists
// twice the sites for about the same per-class cost; at t = 10^4 the two
// are within 2 %.
int choose_pair_segw(uint32_t L) {
    const int nseg = ((int)L + 1024) / 2048 > 0 ? ((int)L + 1024) / 2048 : 1;
    int w = ((int)L / nseg + 31) & ~31;
    const int cap = ((int)L - 64) & ~31;
    if (w > cap) w = cap;
    while (w > 32 && pgg::pair_lds_bytes(w) > pgg::max_dynamic_lds()) w -= 32;
    return w;
}

// Automatic choice between the segment kernel and its paired form: the
// paired launch (two residues) wins when its workgroups are all resident at
// once with one or two per CU (measured: L = 4096, 512 workgroups on 256
// CUs, 3.88e11 against 3.67e11 site updates/s); with fewer workgroups both
// are latency-bound alike, with more the paired launch runs in rounds.
bool pair_fits(const pgg_params* p, int device) {
    if (p->group != 0 || p->L < 512 || p->L % 32 != 0) return false;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        return false;
    const int segw = choose_pair_segw(p->L);
    const long blocks = (long)((p->L + pgg::kPairBand - 1) / pgg::kPairBand) * (long)((p->L + segw - 1) / segw);
    return blocks >= cus && blocks <= 2L * cus && pgg::pair_lds_bytes(segw) <= pgg::max_dynamic_lds();
}

}  // namespace

namespace pgg {
// The automatic single-lattice plan of the segment paths for a bit-packed
// lattice of side L >= 64 (kernel AUTO, group 0): the paired kernel or the
// single-residue one, and the segment width.
void auto_segment_plan(uint32_t L, int device, bool* pair, int* segw) {
    pgg_params p;
    std::memset(&p, 0, sizeof(p));
    p.L = L;
    p.layout = PGG_LAYOUT_BITS;
    *pair = pair_fits(&p, device);
    *segw = *pair ? choose_pair_segw(L) : choose_segw(L, kWavesPerGroup);
}
}  // namespace pgg

namespace {

// The kernel a handle runs (an internal id for the tiled schedule and the
// pairwise game), on `device`.
int choose_kernel(const pgg_params* p, int device) {
    if (p->game == PGG_GAME_PAIRWISE_PD) return kKernelPd;
    if (p->schedule == PGG_SCHEDULE_TILED) return kKernelTiled;
    if (p->kernel != PGG_KERNEL_AUTO) return (int)p->kernel;
    if (p->L < 64) return p->layout == PGG_LAYOUT_INT8 ? PGG_KERNEL_COLOUR : PGG_KERNEL_ROWBAND_COMPACT;
    if (p->L <= kResidentAutoMaxL && pgg::resident_fits((int)p->L) && p->group == 0) return PGG_KERNEL_RESIDENT;
    return pair_fits(p, device) ? PGG_KERNEL_SEGMENT_PAIR : PGG_KERNEL_SEGMENT;
}

bool strip_fits(uint32_t L, uint32_t H) {
    return pgg::strip_lds_bytes((int)L, (int)H, 1) <= pgg::max_dynamic_lds();
}

bool params_valid(const pgg_params* p, const char** why) {
    if (!p) { *why = "params is NULL"; return false; }
    if (p->L < 4 || p->L > 32768 || (p->L % 4) != 0) { *why = "L must be a multiple of 4 in [4, 32768]"; return false; }
    if (!std::isfinite(p->r) || p->r < 0.0) { *why = "r must be finite and >= 0"; return false; }
    if (!std::isfinite(p->K) || !(p->K > 0.0)) { *why = "K must be finite and > 0"; return false; }
    if (!(p->p0 >= 0.0 && p->p0 <= 1.0)) { *why = "p0 must lie in [0, 1]"; return false; }
    if (p->layout != PGG_LAYOUT_INT8 && p->layout != PGG_LAYOUT_BITS) { *why = "unknown layout"; return false; }
    if (p->game != PGG_GAME_PUBLIC_GOODS && p->game != PGG_GAME_PAIRWISE_PD) { *why = "unknown game"; return false; }
    if (p->game == PGG_GAME_PAIRWISE_PD) {
        if (p->schedule != PGG_SCHEDULE_COLOUR16 || p->kernel != PGG_KERNEL_AUTO || p->tile != 0 || p->group != 0) {
            *why = "the pairwise game takes schedule 0 (its own 8-colour sweep), kernel AUTO, tile 0 and group 0";
            return false;
        }
        return true;
    }
    if (p->schedule == PGG_SCHEDULE_TILED) {
        if (p->L % 8 != 0) { *why = "the tiled schedule needs L % 8 == 0"; return false; }
        if (p->kernel != PGG_KERNEL_AUTO || p->tile != 0 || p->group != 0) {
            *why = "the tiled schedule takes kernel AUTO, tile 0 and group 0";
            return false;
        }
        return true;
    }
    if (p->schedule != PGG_SCHEDULE_COLOUR16) { *why = "unknown schedule"; return false; }
    const uint32_t tr = p->tile;
    const bool segment = p->kernel == PGG_KERNEL_SEGMENT || (p->kernel == PGG_KERNEL_AUTO && p->L >= 64);
    if (p->group != 0 && !segment && p->kernel != PGG_KERNEL_RESIDENT) {
        *why = "group applies to the segment and resident kernels only";
        return false;
    }
    switch (p->kernel) {
        case PGG_KERNEL_AUTO:
            if (tr != 0) { *why = "tile needs an explicit kernel"; return false; }
            break;
        case PGG_KERNEL_COLOUR:
            if (p->layout != PGG_LAYOUT_INT8) { *why = "the colour kernel needs the int8 layout"; return false; }
            if (tr != 0) { *why = "the colour kernel takes no tile"; return false; }
            break;
        case PGG_KERNEL_ROWBAND:
        case PGG_KERNEL_ROWBAND_COMPACT:
        case PGG_KERNEL_ROWBAND_STAGED: {
            if (p->layout != PGG_LAYOUT_BITS) { *why = "row-band kernels need the bits layout"; return false; }
            if (tr > p->L / 4) { *why = "tile exceeds the L/4 rows of a residue"; return false; }
            const int R = tr ? (int)tr : choose_R(p->L);
            const size_t lds = p->kernel == PGG_KERNEL_ROWBAND_STAGED
                                   ? pgg::staged_lds_bytes((int)p->L, R)
                                   : pgg::rowband_lds_bytes((int)p->L, R, p->kernel == PGG_KERNEL_ROWBAND_COMPACT);
            if (lds > pgg::max_dynamic_lds()) { *why = "the kernel's LDS footprint does not fit at this L and tile"; return false; }
            break;
        }
        case PGG_KERNEL_SEGMENT: {
            if (p->L < 64) { *why = "the segment kernel needs L >= 64"; return false; }
            if (tr != 0 && !pgg::segw_valid((int)p->L, (int)tr)) { *why = "segment tile must be a multiple of 32 and <= L - 32, or L (whole rows)"; return false; }
            const int wpg = p->group ? (int)p->group : pgg::kWavesPerGroup;
            if (!pgg::ens_wpg_valid(wpg)) { *why = "group must be 0, 2, 4 or 8"; return false; }
            if (segment_lds(p->L, tr ? (int)tr : choose_segw(p->L, wpg), wpg) > pgg::max_dynamic_lds()) {
                *why = "the segment kernel's LDS footprint does not fit at this tile and group";
                return false;
            }
            break;
        }
        case PGG_KERNEL_SEGMENT_PAIR: {
            if (p->L < 512 || p->L % 32 != 0) { *why = "the paired segment kernel needs L >= 512, a multiple of 32"; return false; }
            if (tr != 0 && (tr % 32 != 0 || tr + 64 > p->L)) { *why = "paired segment tile must be a multiple of 32 and <= L - 64"; return false; }
            if (p->group != 0) { *why = "the paired segment kernel takes no group"; return false; }
            if (pgg::pair_lds_bytes(tr ? (int)tr : choose_pair_segw(p->L)) > pgg::max_dynamic_lds()) {
                *why = "the paired segment kernel's LDS footprint does not fit at this tile";
                return false;
            }
            break;
        }
        case PGG_KERNEL_RESIDENT:
            if (!pgg::resident_fits((int)p->L)) { *why = "the resident kernel needs L a multiple of 32 in [64, 512]"; return false; }
            if (tr != 0) { *why = "the resident kernel takes tile 0"; return false; }
            if (p->group != 0 && !pgg::resident_waves_valid((int)p->group)) {
                *why = "the resident kernel's group (waves) must be 0, 4, 8 or 16";
                return false;
            }
            break;
        case PGG_KERNEL_STRIP:
            if (p->layout != PGG_LAYOUT_BITS) { *why = "the strip kernel needs the bits layout"; return false; }
            if (tr != 0 && (tr < 4 || tr > p->L)) { *why = "strip tile must lie in [4, L]"; return false; }
            if (!strip_fits(p->L, tr ? tr : 4)) { *why = "the strip kernel's LDS footprint does not fit at this L"; return false; }
            break;
        default: *why = "unknown kernel"; return false;
    }
    return true;
}

int bits_stride(uint32_t L) { return 2 * (int)((L + 63) / 64); }

size_t lattice_bytes(const pgg_params* p) {
    if (p->layout == PGG_LAYOUT_INT8) return (size_t)p->L * p->L;
    return (size_t)p->L * (size_t)bits_stride(p->L) * sizeof(uint32_t);
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

pgg_status device_fail(pgg_sim* s, hipError_t e, const char* what) {
    set_err("%s: %s", what, hipGetErrorString(e));
    if (s) s->poisoned = true;
    return PGG_E_DEVICE;
}

#define PGG_HIP(s, call)                                       \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return device_fail((s), e_, #call); \
    } while (0)

#define PGG_LIVE(s)                                                           \
    do {                                                                      \
        if (!(s)) { set_err("handle is NULL"); return PGG_E_INVAL; }         \
        if ((s)->poisoned) { set_err("handle poisoned by an earlier device error"); return PGG_E_STATE; } \
    } while (0)

void release(pgg_sim* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    if (s->owns_lattice && s->lattice) (void)hipFree(s->lattice);
    if (s->lattice2) (void)hipFree(s->lattice2);
    if (s->shadow) (void)hipFree(s->shadow);
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipGraph_t g : s->graph_defs) (void)hipGraphDestroy(g);
    if (s->d_rep) (void)hipFree(s->d_rep);
    if (s->d_gdelta) (void)hipFree(s->d_gdelta);
    if (s->d_gcounts) (void)hipFree(s->d_gcounts);
    if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
    if (s->d_table) (void)hipFree(s->d_table);
    if (s->d_nc) (void)hipFree(s->d_nc);
    if (s->d_delta) (void)hipFree(s->d_delta);
    if (s->d_counts) (void)hipFree(s->d_counts);
    if (s->d_drawn) (void)hipFree(s->d_drawn);
    if (s->d_span) (void)hipFree(s->d_span);
    for (hipEvent_t ev : s->chunk_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (s->d_tasks) (void)hipFree(s->d_tasks);
    if (s->d_ring) (void)hipFree(s->d_ring);
    if (s->d_abort) (void)hipFree(s->d_abort);
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    delete s;
}

// Fold the recorded event pairs into the totals (synchronises the stream).
hipError_t fold_timing(pgg_sim* s) {
    if (s->events_used == 0) return hipSuccess;
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return e;
    for (size_t q = 0; q + 1 < s->events_used; q += 2) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, s->events[q], s->events[q + 1]);
        if (e != hipSuccess) return e;
        s->timed_ms += ms;
        s->timed_launches += 1;
    }
    s->events_used = 0;
    return hipSuccess;
}

// Bracket one kernel launch with events when timing is enabled.
template <class F>
hipError_t timed_launch(pgg_sim* s, F&& launch) {
    if (!s->timing) return launch();
    if (s->events_used + 2 > s->events.size()) {
        hipError_t e = fold_timing(s);
        if (e != hipSuccess) return e;
        while (s->events.size() < 8192) {
            hipEvent_t ev;
            e = hipEventCreate(&ev);
            if (e != hipSuccess) return e;
            s->events.push_back(ev);
        }
    }
    hipError_t e = hipEventRecord(s->events[s->events_used], s->stream);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(s->events[s->events_used + 1], s->stream);
    s->events_used += 2;
    return e;
}

// Split the lattice into strips for the persistent kernel: as many strips as
// workgroups can be resident at once (at least 4 rows each, or tile),
// sizes differing by at most one row.
pgg_status plan_strips(pgg_sim* s, uint32_t tile) {
    const int L = (int)s->p.L, nw = (L + 31) / 32;
    int cus = 0, bpc = 0, dev = 0;
    int H = tile ? (int)tile : 4;
    hipError_t e = hipSuccess;
    for (;;) {
        s->strip_lds = pgg::strip_lds_bytes(L, H + 1, 1);  // strips hold H or H + 1 rows
        e = pgg::strip_capacity(s->strip_lds, &bpc, &cus);
        if (e != hipSuccess) { set_err("occupancy query failed: %s", hipGetErrorString(e)); return PGG_E_DEVICE; }
        const int capacity = bpc * cus;
        if (capacity < 1) { set_err("the strip kernel cannot be resident"); return PGG_E_INVAL; }
        const int S = (L + H - 1) / H;
        if (S <= capacity) break;
        if (tile) { set_err("%d strips of %d rows exceed the %d resident workgroups", S, H, capacity); return PGG_E_INVAL; }
        H = (L + capacity - 1) / capacity;
        if (H < 4) H = 4;
    }
    const int S = (L + H - 1) / H;
    const int base = L / S, extra = L % S;
    std::vector<pgg::StripTask> tasks(S);
    int r0 = 0;
    for (int k = 0; k < S; ++k) {
        pgg::StripTask& tk = tasks[k];
        std::memset(&tk, 0, sizeof(tk));
        tk.lat = (uint32_t*)s->lattice;
        tk.T = s->d_table;
        tk.L = L;
        tk.stride = s->stride;
        tk.nw = nw;
        tk.r0 = r0;
        tk.H = base + (k < extra ? 1 : 0);
        tk.up = (k + S - 1) % S;
        tk.down = (k + 1) % S;
        tk.k0 = (uint32_t)s->p.seed;
        tk.k1 = (uint32_t)(s->p.seed >> 32);
        r0 += tk.H;
    }
    s->n_tasks = S;
    s->strip_G = 1;
    s->ring_words = (size_t)S * 2 * 6 * nw;
    int rate_khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate_khz <= 0)
        rate_khz = 100000;
    s->wait_ticks = (uint64_t)rate_khz * 1000ull * 4ull;  // 4 s without neighbour progress
    auto alloc = [&](void** ptr, size_t bytes) -> hipError_t { return hipMalloc(ptr, bytes); };
    if ((e = alloc((void**)&s->d_tasks, S * sizeof(pgg::StripTask))) != hipSuccess ||
        (e = alloc((void**)&s->d_ring, (size_t)S * 2 * 6 * nw * sizeof(uint64_t))) != hipSuccess ||
        (e = alloc((void**)&s->d_abort, sizeof(uint32_t))) != hipSuccess) {
        set_err("hipMalloc failed: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? PGG_E_NOMEM : PGG_E_DEVICE;
    }
    e = hipMemcpyAsync(s->d_tasks, tasks.data(), S * sizeof(pgg::StripTask), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = pgg::launch_fill_u32(s->d_abort, 1, 0u, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) { set_err("strip plan upload failed: %s", hipGetErrorString(e)); return PGG_E_DEVICE; }
    return PGG_OK;
}

// The one-replica descriptors and buffers of the segment kernel.
pgg_status plan_segment_graph(pgg_sim* s) {
    pgg::EnsRep& rp = s->seg_rep;
    std::memset(&rp, 0, sizeof(rp));
    pgg::ens_geometry(rp, (int)s->p.L, s->segw);
    rp.k0 = (uint32_t)s->p.seed;
    rp.k1 = (uint32_t)(s->p.seed >> 32);
    hipError_t e = hipMalloc((void**)&s->d_rep, 2 * sizeof(pgg::EnsRep));
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_gdelta, (size_t)kGraphChunk * pgg::kSweepWords * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_gcounts, (size_t)kGraphChunk * sizeof(unsigned long long));
    // non-blocking: a legacy-stream call of another thread never depends on a capture in progress
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        set_err("segment graph buffers: %s", hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? PGG_E_NOMEM : PGG_E_DEVICE;
    }
    rp.lat = s->shadow ? s->shadow : (uint32_t*)s->lattice;
    rp.lat2 = s->lattice2;
    rp.T = s->d_table;
    rp.delta = s->d_gdelta;
    rp.nc = s->d_nc;
    rp.drawn = nullptr;
    if (s->pair) {
        s->seg_waves = pgg::pair_blocks(rp);  // workgroups of one launch
        s->seg_lds = pgg::pair_lds_bytes(rp.segw);
        s->launches_per_sweep = 2;
    } else {
        s->seg_waves = pgg::ens_waves(rp, s->wpg);
        s->seg_lds = pgg::ens_lds_bytes(pgg::ens_wave_words(rp), s->wpg);
        s->launches_per_sweep = 4;
    }
    const pgg::EnsRep both[2] = {rp, rp};
    e = hipMemcpyAsync(s->d_rep, both, sizeof(both), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) { set_err("segment graph descriptor: %s", hipGetErrorString(e)); return PGG_E_DEVICE; }
    return PGG_OK;
}

// The captured chunk of `len` sweeps (captured on the handle's own capture
// stream -- the null stream cannot be captured -- and launched on its
// stream).  Timing mode has graphs of its own: they run the timing
// descriptor (which counts draws) and record each launch's span.
hipError_t segment_graph(pgg_sim* s, int len, bool timing, hipGraphExec_t* out) {
    const int key = 2 * len + (timing ? 1 : 0);
    auto it = s->graphs.find(key);
    if (it != s->graphs.end()) { *out = it->second; return hipSuccess; }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t enq =
        timing ? pgg::launch_span_reset(s->d_span, s->launches_per_sweep * len, s->capture_stream) : hipSuccess;
    if (enq == hipSuccess && s->pair)
        enq = pgg::launch_pair_chunk(s->d_rep + (timing ? 1 : 0), s->seg_waves, s->seg_lds, len, kGraphChunk,
                                     s->d_gcounts, s->capture_stream, timing ? s->d_span : nullptr);
    else if (enq == hipSuccess)
        enq = pgg::launch_ens_chunk(s->d_rep + (timing ? 1 : 0), 1, s->seg_waves, s->seg_lds, len, kGraphChunk, true,
                                    s->d_gcounts, s->capture_stream, s->wpg, timing ? s->d_span : nullptr);
    e = hipStreamEndCapture(s->capture_stream, &g);
    if (enq != hipSuccess) { if (g) (void)hipGraphDestroy(g); return enq; }
    if (e != hipSuccess) return e;
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return e; }
    s->graph_defs.push_back(g);
    s->graphs[key] = ex;
    e = hipGraphUpload(ex, s->stream);  // device-side setup now, not at the first (possibly timed) launch
    if (e != hipSuccess) return e;
    *out = ex;
    return hipSuccess;
}

// Timing mode, after a chunk of `len` sweeps has completed: add the chunk's
// event time and every launch's span (latest end minus earliest start over
// its records) to the totals.
pgg_status fold_segment_timing(pgg_sim* s, int len) {
    const int nl = s->launches_per_sweep * len;
    std::vector<unsigned long long> span((size_t)nl * pgg::kSpanWords);
    PGG_HIP(s, hipMemcpyAsync(span.data(), s->d_span, span.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                              s->stream));
    PGG_HIP(s, hipStreamSynchronize(s->stream));
    float ms = 0.f;
    PGG_HIP(s, hipEventElapsedTime(&ms, s->chunk_ev[0], s->chunk_ev[1]));
    s->timed_ms += ms;
    s->timed_launches += (uint64_t)nl;
    for (int l = 0; l < nl; ++l) {
        unsigned long long lo = ~0ull, hi = 0ull;
        for (int x = 0; x < pgg::kSpanSlots; ++x) {
            lo = std::min(lo, span[(size_t)pgg::kSpanWords * l + 2 * x]);
            hi = std::max(hi, span[(size_t)pgg::kSpanWords * l + 2 * x + 1]);
        }
        if (lo != ~0ull && hi >= lo) {
            s->span_us += (double)(hi - lo) * 1e3 / s->wall_khz;
            s->span_launches += 1;
        }
    }
    return PGG_OK;
}

// pgg_sweep for the segment kernel: graph replays.  Chunks are kGraphChunk
// sweeps, the rest is split into powers of two, and the graphs of all these
// lengths are captured on the first call of a mode, so no later (timed) call
// instantiates one.  Timing mode synchronises after every chunk.  int8
// layout: the graphs run on the bit-packed working copy, packed from the
// int8 lattice before the first chunk and unpacked into it after the last.
pgg_status sweep_segment(pgg_sim* s, uint32_t n_sweeps, uint64_t* coop_counts) {
    static_assert((kGraphChunk & (kGraphChunk - 1)) == 0, "kGraphChunk must be a power of two");
    const bool timing = s->timing;
    for (int len = kGraphChunk; len >= 1; len >>= 1) {
        hipGraphExec_t g = nullptr;
        PGG_HIP(s, segment_graph(s, len, timing, &g));
    }
    PGG_HIP(s, pgg::launch_ens_set_t0(s->d_rep + (timing ? 1 : 0), 1, (uint32_t)s->t, s->stream));
    if (s->shadow)
        PGG_HIP(s, pgg::launch_pack((const uint8_t*)s->lattice, s->shadow, (int)s->p.L, s->stride, s->stream));
    uint32_t done = 0;
    while (done < n_sweeps) {
        const uint32_t rem = n_sweeps - done;
        const int len = rem >= (uint32_t)kGraphChunk ? kGraphChunk : (int)(1u << (31 - __builtin_clz(rem)));
        hipGraphExec_t g = nullptr;
        PGG_HIP(s, segment_graph(s, len, timing, &g));
        if (timing) PGG_HIP(s, hipEventRecord(s->chunk_ev[0], s->stream));
        PGG_HIP(s, hipGraphLaunch(g, s->stream));
        if (timing) PGG_HIP(s, hipEventRecord(s->chunk_ev[1], s->stream));
        if (coop_counts)
            PGG_HIP(s, hipMemcpyAsync(coop_counts + done, s->d_gcounts, (size_t)len * sizeof(uint64_t),
                                      hipMemcpyDeviceToHost, s->stream));
        if (timing) {
            PGG_HIP(s, hipStreamSynchronize(s->stream));
            pgg_status fs = fold_segment_timing(s, len);
            if (fs != PGG_OK) return fs;
        }
        done += (uint32_t)len;
    }
    if (s->shadow)
        PGG_HIP(s, pgg::launch_unpack(s->shadow, (uint8_t*)s->lattice, (int)s->p.L, s->stride, s->stream));
    if (coop_counts) PGG_HIP(s, hipStreamSynchronize(s->stream));
    s->t += n_sweeps;
    return PGG_OK;
}

// After a stream synchronisation: a persistent launch that gave up waiting
// leaves the abort flag set; report it and poison the handle.
pgg_status check_abort(pgg_sim* s) {
    if (!s->d_abort) return PGG_OK;
    uint32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, s->d_abort, sizeof(v), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return device_fail(s, e, "abort flag read");
    if (v) {
        set_err("a persistent strip launch aborted: a workgroup waited too long for its neighbours");
        s->poisoned = true;
        return PGG_E_DEVICE;
    }
    return PGG_OK;
}

}  // namespace

extern "C" {

const char* pgg_last_error(void) { return g_err; }

size_t pgg_device_bytes(const pgg_params* p) {
    const char* why = nullptr;
    if (!params_valid(p, &why)) return 0;
    return lattice_bytes(p);
}

pgg_status pgg_plan(const pgg_params* p, uint32_t* kernel, uint32_t* tile) {
    if (!kernel || !tile) { set_err("NULL argument"); return PGG_E_INVAL; }
    const char* why = nullptr;
    if (!params_valid(p, &why)) { set_err("invalid parameters: %s", why); return PGG_E_INVAL; }
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) { set_err("no HIP device"); return PGG_E_DEVICE; }
    const int k = choose_kernel(p, device);
    const int wpg = p->group ? (int)p->group : pgg::kWavesPerGroup;
    uint32_t w = 0;
    switch (k) {
        case PGG_KERNEL_SEGMENT: w = p->tile ? p->tile : (uint32_t)choose_segw(p->L, wpg); break;
        case PGG_KERNEL_SEGMENT_PAIR: w = p->tile ? p->tile : (uint32_t)choose_pair_segw(p->L); break;
        case PGG_KERNEL_ROWBAND:
        case PGG_KERNEL_ROWBAND_COMPACT:
        case PGG_KERNEL_ROWBAND_STAGED: w = p->tile ? p->tile : (uint32_t)choose_R(p->L); break;
        case PGG_KERNEL_RESIDENT: w = p->group ? p->group : (uint32_t)pgg::resident_auto_waves((int)p->L); break;
        case PGG_KERNEL_STRIP: w = p->tile; break;
        default: w = 0;
    }
    *kernel = (k == kKernelPd || k == kKernelTiled) ? (uint32_t)PGG_KERNEL_AUTO : (uint32_t)k;
    *tile = w;
    return PGG_OK;
}

pgg_status pgg_init(const pgg_params* p, void* dev_buf, size_t dev_bytes, void* hip_stream,
                    pgg_sim** out) {
    g_err[0] = 0;
    if (!out) { set_err("out is NULL"); return PGG_E_INVAL; }
    *out = nullptr;
    const char* why = nullptr;
    if (!params_valid(p, &why)) { set_err("invalid parameters: %s", why); return PGG_E_INVAL; }
    if (dev_buf && ((uintptr_t)dev_buf & 3u) != 0) {
        set_err("dev_buf must be 4-byte aligned");
        return PGG_E_INVAL;
    }
    if (dev_buf && dev_bytes < lattice_bytes(p)) {
        set_err("dev_buf holds %zu bytes, the lattice needs %zu", dev_bytes, lattice_bytes(p));
        return PGG_E_INVAL;
    }
    pgg_sim* s = new (std::nothrow) pgg_sim();
    if (!s) { set_err("host allocation failed"); return PGG_E_NOMEM; }
    s->p = *p;
    s->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&s->device) != hipSuccess) {
        set_err("no HIP device");
        delete s;
        return PGG_E_DEVICE;
    }
    s->stride = bits_stride(p->L);
    s->R = p->tile ? (int)p->tile : choose_R(p->L);
    s->kernel = choose_kernel(p, s->device);
    s->wpg = p->group ? (int)p->group : pgg::kWavesPerGroup;
    if (s->kernel == PGG_KERNEL_SEGMENT) s->segw = p->tile ? (int)p->tile : choose_segw(p->L, s->wpg);
    if (s->kernel == PGG_KERNEL_SEGMENT_PAIR) {
        s->segw = p->tile ? (int)p->tile : choose_pair_segw(p->L);
        s->pair = true;
    }
    const bool segment_path = s->kernel == PGG_KERNEL_SEGMENT || s->kernel == PGG_KERNEL_SEGMENT_PAIR;

    auto alloc = [&](void** ptr, size_t bytes) -> pgg_status {
        hipError_t e = hipMalloc(ptr, bytes);
        if (e != hipSuccess) {
            set_err("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? PGG_E_NOMEM : PGG_E_DEVICE;
        }
        return PGG_OK;
    };
    pgg_status st = PGG_OK;
    if (dev_buf) {
        s->lattice = dev_buf;
    } else {
        st = alloc(&s->lattice, lattice_bytes(p));
        s->owns_lattice = (st == PGG_OK);
    }
    if (st == PGG_OK) st = alloc((void**)&s->d_table, pgg::kTableSize * sizeof(uint32_t));
    if (st == PGG_OK) st = alloc((void**)&s->d_nc, sizeof(unsigned long long));
    if (st == PGG_OK && s->kernel == PGG_KERNEL_STRIP) st = plan_strips(s, p->tile);
    pgg_params bits = *p;
    bits.layout = PGG_LAYOUT_BITS;
    const bool packed_copy =
        (segment_path || s->kernel == kKernelTiled || s->kernel == kKernelPd || s->kernel == PGG_KERNEL_RESIDENT) &&
        p->layout == PGG_LAYOUT_INT8;
    if (st == PGG_OK && packed_copy) st = alloc((void**)&s->shadow, lattice_bytes(&bits));
    if (st == PGG_OK && segment_path) st = alloc((void**)&s->lattice2, lattice_bytes(&bits));
    if (st == PGG_OK && segment_path) st = plan_segment_graph(s);
    if (st != PGG_OK) { release(s); return st; }

    if (s->kernel == kKernelPd) {
        std::memset(s->h_table, 0, sizeof(s->h_table));
        pgg::pd_table(p->r, p->K, s->h_table);
    } else {
        pgg::fermi_table(p->r, p->K, s->h_table);
    }
    hipError_t e = pgg::upload_table(s->h_table, s->d_table, s->stream);
    if (e == hipSuccess)
        e = pgg::launch_init((int)p->layout, s->lattice, (int)p->L, s->stride, p->p0, p->seed, s->d_nc,
                             s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        set_err("initialisation failed: %s", hipGetErrorString(e));
        release(s);
        return PGG_E_DEVICE;
    }
    *out = s;
    return PGG_OK;
}

namespace {
// Make d_delta / d_counts hold n sweeps (n <= kChunk).  Work already queued
// on the stream may still use the old buffers, so the stream is drained
// before they are freed.
pgg_status grow_delta(pgg_sim* s, uint32_t n) {
    if (n <= s->delta_sweeps) return PGG_OK;
    if (s->d_delta || s->d_counts) {
        const hipError_t e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return device_fail(s, e, "hipStreamSynchronize");
        if (s->d_delta) (void)hipFree(s->d_delta);
        if (s->d_counts) (void)hipFree(s->d_counts);
        s->d_delta = nullptr;
        s->d_counts = nullptr;
        s->delta_sweeps = 0;
    }
    hipError_t e = hipMalloc((void**)&s->d_delta, (size_t)n * pgg::kSweepWords * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_counts, (size_t)n * sizeof(unsigned long long));
    if (e != hipSuccess) {
        set_err("hipMalloc of the per-sweep counters (%u sweeps) failed: %s", n, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? PGG_E_NOMEM : PGG_E_DEVICE;
    }
    s->delta_sweeps = n;
    return PGG_OK;
}
}  // namespace

pgg_status pgg_sweep(pgg_sim* s, uint32_t n_sweeps, uint64_t* coop_counts) {
    PGG_LIVE(s);
    if (s->t + (uint64_t)n_sweeps > 4294967296ull) {
        set_err("sweep index would exceed 2^32");
        return PGG_E_INVAL;
    }
    if (n_sweeps == 0) return PGG_OK;
    DeviceGuard guard(s->device);
    if (s->kernel == PGG_KERNEL_SEGMENT || s->kernel == PGG_KERNEL_SEGMENT_PAIR)
        return sweep_segment(s, n_sweeps, coop_counts);
    const int L = (int)s->p.L;
    // the tiled schedule and the resident kernel sweep a bit-packed working
    // copy of an int8 lattice
    uint32_t* tiled_lat = s->shadow ? s->shadow : (uint32_t*)s->lattice;
    if (s->shadow)
        PGG_HIP(s, pgg::launch_pack((const uint8_t*)s->lattice, s->shadow, L, s->stride, s->stream));
    {
        const pgg_status gs = grow_delta(s, std::min(kChunk, n_sweeps));
        if (gs != PGG_OK) return gs;
    }
    uint32_t done = 0;
    while (done < n_sweeps) {
        const uint32_t n = std::min(kChunk, n_sweeps - done);
        PGG_HIP(s, pgg::launch_fill_u64(s->d_delta, (int64_t)n * pgg::kSweepWords, 0ull, s->stream));
        if (s->kernel == PGG_KERNEL_STRIP) {
            const uint32_t t0 = (uint32_t)(s->t + done);
            PGG_HIP(s, pgg::launch_tasks_set(s->d_tasks, s->n_tasks, t0, (int)n, s->d_delta,
                                             s->timing ? s->d_drawn : nullptr, s->stream));
            // ring tags start at 0 in every launch (tags are step + 1 >= 1)
            PGG_HIP(s, pgg::launch_fill_u64((unsigned long long*)s->d_ring, (int64_t)s->ring_words, 0ull, s->stream));
            PGG_HIP(s, timed_launch(s, [&] {
                return pgg::launch_strip(s->d_tasks, s->n_tasks, s->d_ring, s->d_abort, s->wait_ticks,
                                         s->strip_G, s->strip_lds, s->stream);
            }));
        }
        if (s->kernel == PGG_KERNEL_RESIDENT) {
            const uint32_t t0 = (uint32_t)(s->t + done);
            const int W = s->p.group ? (int)s->p.group : pgg::resident_auto_waves(L);
            PGG_HIP(s, timed_launch(s, [&] {
                return pgg::launch_resident(tiled_lat, L, s->stride, W, t0, (int)n, s->p.seed, s->d_table,
                                            s->d_delta, s->timing ? s->d_drawn : nullptr, s->stream);
            }));
        }
        const bool per_sweep = s->kernel != PGG_KERNEL_STRIP && s->kernel != PGG_KERNEL_RESIDENT;
        for (uint32_t q = 0; per_sweep && q < n; ++q) {
            const uint32_t t = (uint32_t)(s->t + done + q);
            unsigned long long* dq = s->d_delta + (size_t)q * pgg::kSweepWords;
            if (s->kernel == kKernelPd) {
                for (int k = 0; k < 8; ++k)
                    PGG_HIP(s, timed_launch(s, [&] {
                        return pgg::launch_pd_class(tiled_lat, L, s->stride, k, t, s->p.seed, s->d_table, dq,
                                                    s->stream);
                    }));
            } else if (s->kernel == kKernelTiled) {
                for (int part = 0; part < 4; ++part)
                    PGG_HIP(s, timed_launch(s, [&] {
                        return pgg::launch_tiled_part(tiled_lat, L, s->stride, part, t, s->p.seed,
                                                      s->d_table, dq, s->stream);
                    }));
            } else if (s->kernel == PGG_KERNEL_COLOUR) {
                for (int k = 0; k < 16; ++k)
                    PGG_HIP(s, timed_launch(s, [&] {
                        return pgg::launch_colour_phase((uint8_t*)s->lattice, L, k, t, s->p.seed,
                                                        s->d_table, dq, s->stream);
                    }));
            } else if (s->kernel == PGG_KERNEL_ROWBAND_STAGED) {
                unsigned long long* drawn = s->timing ? s->d_drawn : nullptr;
                for (int a = 0; a < 4; ++a)
                    PGG_HIP(s, timed_launch(s, [&] {
                        return pgg::launch_staged_residue((uint32_t*)s->lattice, L, s->stride, s->R, a, t,
                                                          s->p.seed, s->d_table, dq, drawn, s->stream);
                    }));
            } else {
                const bool compact = s->kernel == PGG_KERNEL_ROWBAND_COMPACT;
                unsigned long long* drawn = s->timing ? s->d_drawn : nullptr;
                for (int a = 0; a < 4; ++a)
                    PGG_HIP(s, timed_launch(s, [&] {
                        return pgg::launch_rowband_residue((uint32_t*)s->lattice, L, s->stride, s->R,
                                                           compact, a, t, s->p.seed, s->d_table, dq,
                                                           drawn, s->stream);
                    }));
            }
        }
        PGG_HIP(s, pgg::launch_scan_counts(s->d_delta, s->d_counts, (int)n, s->d_nc, s->stream));
        if (coop_counts) {
            PGG_HIP(s, hipMemcpyAsync(coop_counts + done, s->d_counts, n * sizeof(uint64_t),
                                      hipMemcpyDeviceToHost, s->stream));
            PGG_HIP(s, hipStreamSynchronize(s->stream));
            pgg_status as = check_abort(s);
            if (as != PGG_OK) return as;
        }
        done += n;
    }
    if (s->shadow)
        PGG_HIP(s, pgg::launch_unpack(s->shadow, (uint8_t*)s->lattice, L, s->stride, s->stream));
    s->t += n_sweeps;
    return PGG_OK;
}

pgg_status pgg_coop_count(pgg_sim* s, uint64_t* n_c) {
    PGG_LIVE(s);
    if (!n_c) { set_err("n_c is NULL"); return PGG_E_INVAL; }
    DeviceGuard guard(s->device);
    unsigned long long v = 0;
    PGG_HIP(s, hipMemcpyAsync(&v, s->d_nc, sizeof(v), hipMemcpyDeviceToHost, s->stream));
    PGG_HIP(s, hipStreamSynchronize(s->stream));
    pgg_status as = check_abort(s);
    if (as != PGG_OK) return as;
    *n_c = v;
    return PGG_OK;
}

pgg_status pgg_density(pgg_sim* s, double* rho) {
    if (!rho) { set_err("rho is NULL"); return PGG_E_INVAL; }
    uint64_t nc = 0;
    pgg_status st = pgg_coop_count(s, &nc);
    if (st != PGG_OK) return st;
    *rho = (double)nc / ((double)s->p.L * (double)s->p.L);
    return PGG_OK;
}

pgg_status pgg_sweep_index(const pgg_sim* s, uint64_t* t) {
    if (!s || !t) { set_err("NULL argument"); return PGG_E_INVAL; }
    *t = s->t;
    return PGG_OK;
}

pgg_status pgg_read_lattice(pgg_sim* s, uint8_t* host_LxL) {
    PGG_LIVE(s);
    if (!host_LxL) { set_err("host_LxL is NULL"); return PGG_E_INVAL; }
    DeviceGuard guard(s->device);
    const size_t n = (size_t)s->p.L * s->p.L;
    if (s->p.layout == PGG_LAYOUT_INT8) {
        PGG_HIP(s, hipMemcpyAsync(host_LxL, s->lattice, n, hipMemcpyDeviceToHost, s->stream));
        PGG_HIP(s, hipStreamSynchronize(s->stream));
        return check_abort(s);
    }
    uint8_t* tmp = nullptr;
    hipError_t e = hipMalloc((void**)&tmp, n);
    if (e != hipSuccess) { set_err("staging allocation failed: %s", hipGetErrorString(e)); return PGG_E_NOMEM; }
    e = pgg::launch_unpack((const uint32_t*)s->lattice, tmp, (int)s->p.L, s->stride, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host_LxL, tmp, n, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return device_fail(s, e, "read_lattice");
    return check_abort(s);
}

pgg_status pgg_write_lattice(pgg_sim* s, const uint8_t* host_LxL, uint64_t t) {
    PGG_LIVE(s);
    if (!host_LxL) { set_err("host_LxL is NULL"); return PGG_E_INVAL; }
    if (t > 4294967296ull) { set_err("t must be <= 2^32"); return PGG_E_INVAL; }
    const size_t n = (size_t)s->p.L * s->p.L;
    for (size_t x = 0; x < n; ++x)
        if (host_LxL[x] > 1) { set_err("lattice byte %zu is %u, not 0 or 1", x, host_LxL[x]); return PGG_E_INVAL; }
    DeviceGuard guard(s->device);
    if (s->p.layout == PGG_LAYOUT_INT8) {
        PGG_HIP(s, hipMemcpyAsync(s->lattice, host_LxL, n, hipMemcpyHostToDevice, s->stream));
    } else {
        uint8_t* tmp = nullptr;
        hipError_t e = hipMalloc((void**)&tmp, n);
        if (e != hipSuccess) { set_err("staging allocation failed: %s", hipGetErrorString(e)); return PGG_E_NOMEM; }
        e = hipMemcpyAsync(tmp, host_LxL, n, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = pgg::launch_pack(tmp, (uint32_t*)s->lattice, (int)s->p.L, s->stride, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        (void)hipFree(tmp);
        if (e != hipSuccess) return device_fail(s, e, "write_lattice");
    }
    PGG_HIP(s, pgg::launch_count((int)s->p.layout, s->lattice, (int)s->p.L, s->stride, s->d_nc, s->stream));
    PGG_HIP(s, hipStreamSynchronize(s->stream));
    s->t = t;
    return PGG_OK;
}

pgg_status pgg_threshold_table(pgg_sim* s, uint32_t* host_T) {
    PGG_LIVE(s);
    if (!host_T) { set_err("host_T is NULL"); return PGG_E_INVAL; }
    DeviceGuard guard(s->device);
    PGG_HIP(s, hipMemcpyAsync(host_T, s->d_table, pgg::kTableSize * sizeof(uint32_t),
                              hipMemcpyDeviceToHost, s->stream));
    PGG_HIP(s, hipStreamSynchronize(s->stream));
    return PGG_OK;
}

pgg_status pgg_fermi_table(double r, double K, uint32_t* host_T) {
    if (!host_T) { set_err("host_T is NULL"); return PGG_E_INVAL; }
    if (!std::isfinite(r) || r < 0.0) { set_err("r must be finite and >= 0"); return PGG_E_INVAL; }
    if (!std::isfinite(K) || !(K > 0.0)) { set_err("K must be finite and > 0"); return PGG_E_INVAL; }
    pgg::fermi_table(r, K, host_T);
    return PGG_OK;
}

pgg_status pgg_pd_table(double b, double K, uint32_t* host_T) {
    if (!host_T) { set_err("host_T is NULL"); return PGG_E_INVAL; }
    if (!std::isfinite(b) || b < 0.0) { set_err("b must be finite and >= 0"); return PGG_E_INVAL; }
    if (!std::isfinite(K) || !(K > 0.0)) { set_err("K must be finite and > 0"); return PGG_E_INVAL; }
    pgg::pd_table(b, K, host_T);
    return PGG_OK;
}

pgg_status pgg_set_kernel_timing(pgg_sim* s, int enable) {
    PGG_LIVE(s);
    DeviceGuard guard(s->device);
    if (enable && !s->d_drawn) {
        hipError_t e = hipMalloc((void**)&s->d_drawn, pgg::kSweepWords * sizeof(unsigned long long));
        if (e != hipSuccess) { set_err("hipMalloc failed: %s", hipGetErrorString(e)); return PGG_E_NOMEM; }
    }
    if (enable && s->d_rep && !s->d_span) {
        hipError_t e = hipMalloc((void**)&s->d_span, (size_t)kGraphChunk * 4 * pgg::kSpanWords * sizeof(unsigned long long));
        if (e != hipSuccess) { set_err("hipMalloc failed: %s", hipGetErrorString(e)); return PGG_E_NOMEM; }
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device) != hipSuccess || khz <= 0)
            khz = 100000;
        s->wall_khz = (double)khz;
        for (hipEvent_t& ev : s->chunk_ev)
            if (!ev) PGG_HIP(s, hipEventCreate(&ev));
    }
    PGG_HIP(s, fold_timing(s));
    if (enable) PGG_HIP(s, pgg::launch_fill_u64(s->d_drawn, pgg::kSweepWords, 0ull, s->stream));
    if (enable && s->d_rep) {  // the timing descriptor of the segment kernel counts draws
        pgg::EnsRep rp = s->seg_rep;
        rp.drawn = s->d_drawn;
        PGG_HIP(s, hipMemcpyAsync(s->d_rep + 1, &rp, sizeof(rp), hipMemcpyHostToDevice, s->stream));
    }
    PGG_HIP(s, hipStreamSynchronize(s->stream));
    s->timing = enable != 0;
    s->timed_launches = 0;
    s->timed_ms = 0.0;
    s->span_launches = 0;
    s->span_us = 0.0;
    return PGG_OK;
}

pgg_status pgg_kernel_timing(pgg_sim* s, uint64_t* launches, double* total_ms, uint64_t* drawn) {
    PGG_LIVE(s);
    if (!launches || !total_ms || !drawn) { set_err("NULL argument"); return PGG_E_INVAL; }
    DeviceGuard guard(s->device);
    PGG_HIP(s, fold_timing(s));
    unsigned long long d = 0;
    if (s->d_drawn) {
        std::vector<unsigned long long> h(pgg::kSweepWords);
        PGG_HIP(s, hipMemcpyAsync(h.data(), s->d_drawn, h.size() * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, s->stream));
        PGG_HIP(s, hipStreamSynchronize(s->stream));
        for (int k = 0; k < pgg::kSlots; ++k) d += h[(size_t)k * pgg::kSlotStride];
    }
    pgg_status as = check_abort(s);
    if (as != PGG_OK) return as;
    *launches = s->timed_launches;
    *total_ms = s->timed_ms;
    *drawn = d;
    return PGG_OK;
}

pgg_status pgg_kernel_span(pgg_sim* s, uint64_t* launches, double* total_us) {
    PGG_LIVE(s);
    if (!launches || !total_us) { set_err("NULL argument"); return PGG_E_INVAL; }
    *launches = s->span_launches;
    *total_us = s->span_us;
    return PGG_OK;
}

pgg_status pgg_set_strip_wait(pgg_sim* s, double seconds) {
    PGG_LIVE(s);
    if (!(seconds >= 0.0 && seconds <= 3600.0)) { set_err("seconds must lie in [0, 3600]"); return PGG_E_INVAL; }
    int dev = s->device, rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate_khz <= 0)
        rate_khz = 100000;
    s->wait_ticks = (uint64_t)(seconds * (double)rate_khz * 1000.0);
    return PGG_OK;
}

void pgg_destroy(pgg_sim* s) {
    if (!s) return;
    DeviceGuard guard(s->device);
    release(s);
}

}  // extern "C"
