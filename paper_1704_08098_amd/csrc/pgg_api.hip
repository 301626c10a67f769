// C ABI of the engine: validation, ownership, streams and error reporting
// around the kernels.  Declarations and the contract are in include/pgg.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
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

constexpr uint32_t kChunk = 65536;  // sweeps per count-history chunk

}  // namespace

struct pgg_sim {
    pgg_params p;
    hipStream_t stream = nullptr;
    int device = 0;
    void* lattice = nullptr;
    bool owns_lattice = false;
    int stride = 0;  // bits layout: 32-bit words per row
    int kernel = PGG_KERNEL_COLOUR;
    int R = 1;       // rows per workgroup (row-band kernels)
    uint32_t* d_table = nullptr;
    unsigned long long* d_nc = nullptr;
    unsigned long long* d_delta = nullptr;
    unsigned long long* d_counts = nullptr;
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

bool params_valid(const pgg_params* p, const char** why) {
    if (!p) { *why = "params is NULL"; return false; }
    if (p->L < 4 || p->L > 32768 || (p->L % 4) != 0) { *why = "L must be a multiple of 4 in [4, 32768]"; return false; }
    if (!std::isfinite(p->r) || p->r < 0.0) { *why = "r must be finite and >= 0"; return false; }
    if (!std::isfinite(p->K) || !(p->K > 0.0)) { *why = "K must be finite and > 0"; return false; }
    if (!(p->p0 >= 0.0 && p->p0 <= 1.0)) { *why = "p0 must lie in [0, 1]"; return false; }
    if (p->layout != PGG_LAYOUT_INT8 && p->layout != PGG_LAYOUT_BITS) { *why = "unknown layout"; return false; }
    switch (p->kernel) {
        case PGG_KERNEL_AUTO: break;
        case PGG_KERNEL_COLOUR:
            if (p->layout != PGG_LAYOUT_INT8) { *why = "the colour kernel needs the int8 layout"; return false; }
            break;
        case PGG_KERNEL_ROWBAND:
        case PGG_KERNEL_ROWBAND_COMPACT:
        case PGG_KERNEL_ROWBAND_STAGED:
            if (p->layout != PGG_LAYOUT_BITS) { *why = "row-band kernels need the bits layout"; return false; }
            if (p->kernel == PGG_KERNEL_ROWBAND_STAGED && p->L >= 4 && p->L <= 32768 && p->L % 4 == 0 &&
                pgg::staged_lds_bytes((int)p->L, choose_R(p->L)) > pgg::kMaxDynamicLds) {
                *why = "the staged kernel's LDS footprint does not fit at this L"; return false;
            }
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
    if (s->d_table) (void)hipFree(s->d_table);
    if (s->d_nc) (void)hipFree(s->d_nc);
    if (s->d_delta) (void)hipFree(s->d_delta);
    if (s->d_counts) (void)hipFree(s->d_counts);
    if (s->d_drawn) (void)hipFree(s->d_drawn);
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

}  // namespace

extern "C" {

const char* pgg_last_error(void) { return g_err; }

size_t pgg_device_bytes(const pgg_params* p) {
    const char* why = nullptr;
    if (!params_valid(p, &why)) return 0;
    return lattice_bytes(p);
}

pgg_status pgg_init(const pgg_params* p, void* dev_buf, size_t dev_bytes, void* hip_stream,
                    pgg_sim** out) {
    g_err[0] = 0;
    if (!out) { set_err("out is NULL"); return PGG_E_INVAL; }
    *out = nullptr;
    const char* why = nullptr;
    if (!params_valid(p, &why)) { set_err("invalid parameters: %s", why); return PGG_E_INVAL; }
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
    s->R = choose_R(p->L);
    if (p->kernel != PGG_KERNEL_AUTO)
        s->kernel = (int)p->kernel;
    else if (p->layout == PGG_LAYOUT_INT8)
        s->kernel = PGG_KERNEL_COLOUR;
    else
        s->kernel = pgg::staged_lds_bytes((int)p->L, s->R) <= pgg::kMaxDynamicLds ? PGG_KERNEL_ROWBAND_STAGED
                                                                                 : PGG_KERNEL_ROWBAND_COMPACT;

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
    if (st == PGG_OK) st = alloc((void**)&s->d_delta, kChunk * sizeof(unsigned long long));
    if (st == PGG_OK) st = alloc((void**)&s->d_counts, kChunk * sizeof(unsigned long long));
    if (st != PGG_OK) { release(s); return st; }

    hipError_t e = pgg::launch_build_table(p->r, p->K, s->d_table, s->stream);
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

pgg_status pgg_sweep(pgg_sim* s, uint32_t n_sweeps, uint64_t* coop_counts) {
    PGG_LIVE(s);
    if (s->t + (uint64_t)n_sweeps > 4294967296ull) {
        set_err("sweep index would exceed 2^32");
        return PGG_E_INVAL;
    }
    if (n_sweeps == 0) return PGG_OK;
    DeviceGuard guard(s->device);
    const int L = (int)s->p.L;
    uint32_t done = 0;
    while (done < n_sweeps) {
        const uint32_t n = std::min(kChunk, n_sweeps - done);
        PGG_HIP(s, pgg::launch_fill_u64(s->d_delta, n, 0ull, s->stream));
        for (uint32_t q = 0; q < n; ++q) {
            const uint32_t t = (uint32_t)(s->t + done + q);
            unsigned long long* dq = s->d_delta + q;
            if (s->kernel == PGG_KERNEL_COLOUR) {
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
        }
        done += n;
    }
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
        return PGG_OK;
    }
    uint8_t* tmp = nullptr;
    hipError_t e = hipMalloc((void**)&tmp, n);
    if (e != hipSuccess) { set_err("staging allocation failed: %s", hipGetErrorString(e)); return PGG_E_NOMEM; }
    e = pgg::launch_unpack((const uint32_t*)s->lattice, tmp, (int)s->p.L, s->stride, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host_LxL, tmp, n, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return device_fail(s, e, "read_lattice");
    return PGG_OK;
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

pgg_status pgg_set_kernel_timing(pgg_sim* s, int enable) {
    PGG_LIVE(s);
    DeviceGuard guard(s->device);
    if (enable && !s->d_drawn) {
        hipError_t e = hipMalloc((void**)&s->d_drawn, sizeof(unsigned long long));
        if (e != hipSuccess) { set_err("hipMalloc failed: %s", hipGetErrorString(e)); return PGG_E_NOMEM; }
    }
    PGG_HIP(s, fold_timing(s));
    if (enable) PGG_HIP(s, pgg::launch_fill_u64(s->d_drawn, 1, 0ull, s->stream));
    PGG_HIP(s, hipStreamSynchronize(s->stream));
    s->timing = enable != 0;
    s->timed_launches = 0;
    s->timed_ms = 0.0;
    return PGG_OK;
}

pgg_status pgg_kernel_timing(pgg_sim* s, uint64_t* launches, double* total_ms, uint64_t* drawn) {
    PGG_LIVE(s);
    if (!launches || !total_ms || !drawn) { set_err("NULL argument"); return PGG_E_INVAL; }
    DeviceGuard guard(s->device);
    PGG_HIP(s, fold_timing(s));
    unsigned long long d = 0;
    if (s->d_drawn) {
        PGG_HIP(s, hipMemcpyAsync(&d, s->d_drawn, sizeof(d), hipMemcpyDeviceToHost, s->stream));
        PGG_HIP(s, hipStreamSynchronize(s->stream));
    }
    *launches = s->timed_launches;
    *total_ms = s->timed_ms;
    *drawn = d;
    return PGG_OK;
}

void pgg_destroy(pgg_sim* s) {
    if (!s) return;
    DeviceGuard guard(s->device);
    release(s);
}

}  // extern "C"
