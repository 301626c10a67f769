// pgg_sweep_static: the sweep of pgg_sweep on a caller's bit-packed lattice
// with no allocation at all.  The kernels are those of the handle path (the
// segment kernel or its paired form, chosen as pgg_init's AUTO does); every
// buffer they need beyond the caller's lattice and counts -- the replica
// descriptor, the Fermi thresholds, the per-sweep counters, the second
// lattice buffer of the out-of-place sweep and, without caller counts, a
// count buffer -- lives in one file-scope device array, `scratch`, of fixed
// size.  Host code never passes `scratch` itself to a kernel: on the host
// that name is only a stand-in.  Its device address is looked up once per
// device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "pgg.h"
#include "pgg_internal.hpp"

namespace {

// Largest side the scratch holds (the second lattice buffer of L rows of
// 2 ceil(L/64) words), and sweeps per eager chunk.
constexpr uint32_t kStaticMaxL = 4096;
constexpr int kStaticChunk = 64;

constexpr size_t kOffRep = 0;                                  // EnsRep
constexpr size_t kOffTable = 256;                              // 153 thresholds
constexpr size_t kOffNc = 1024;                                // N_C
constexpr size_t kOffCounts = 1280;                            // kStaticChunk counts (no caller counts)
constexpr size_t kOffDelta = 4096;                             // kStaticChunk x kSweepWords
constexpr size_t kOffLat2 = kOffDelta + (size_t)kStaticChunk * pgg::kSweepWords * sizeof(unsigned long long);
constexpr size_t kLat2Bytes = (size_t)kStaticMaxL * (2 * ((kStaticMaxL + 63) / 64)) * sizeof(uint32_t);
constexpr size_t kScratchBytes = kOffLat2 + kLat2Bytes;
static_assert(sizeof(pgg::EnsRep) <= kOffTable - kOffRep, "descriptor slot too small");
static_assert(pgg::kTableSize * sizeof(uint32_t) <= kOffNc - kOffTable, "table slot too small");
static_assert(kOffCounts + kStaticChunk * sizeof(unsigned long long) <= kOffDelta, "counts slot too small");
static_assert(kOffLat2 % 256 == 0, "lattice slot must stay 256-byte aligned");

}  // namespace

// One copy per device, kept until the process ends.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct TableArg {
    uint32_t T[pgg::kTableSize];
};

// The descriptor and the thresholds travel as kernel arguments, so that no
// host memory is read by a copy (a caller may capture the calls in a graph).
__global__ void k_static_setup(pgg::EnsRep* rep_dst, pgg::EnsRep rep, uint32_t* T_dst, TableArg tab) {
    if (threadIdx.x == 0) *rep_dst = rep;
    for (int k = threadIdx.x; k < pgg::kTableSize; k += blockDim.x) T_dst[k] = tab.T[k];
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up once per device).
hipError_t scratch_address(int device, unsigned char** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = (unsigned char*)ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t pgg_sweep_static_scratch_bytes(void) { return kScratchBytes; }

pgg_status pgg_sweep_static(const pgg_params* p, void* dev_lattice, uint64_t t0, uint32_t n_sweeps,
                            uint64_t* dev_counts, void* hip_stream) {
    if (!p || !dev_lattice) { pgg::set_errorf("params or dev_lattice is NULL"); return PGG_E_INVAL; }
    if (p->L < 64 || p->L > kStaticMaxL || p->L % 4 != 0) {
        pgg::set_errorf("pgg_sweep_static: L must be a multiple of 4 in [64, %u] (the scratch holds %zu bytes)",
                        kStaticMaxL, kScratchBytes);
        return PGG_E_INVAL;
    }
    if (!std::isfinite(p->r) || p->r < 0.0) { pgg::set_errorf("r must be finite and >= 0"); return PGG_E_INVAL; }
    if (!std::isfinite(p->K) || !(p->K > 0.0)) { pgg::set_errorf("K must be finite and > 0"); return PGG_E_INVAL; }
    if (p->layout != PGG_LAYOUT_BITS || p->kernel != PGG_KERNEL_AUTO || p->tile != 0 || p->group != 0 ||
        p->schedule != PGG_SCHEDULE_COLOUR16 || p->game != PGG_GAME_PUBLIC_GOODS) {
        pgg::set_errorf("pgg_sweep_static takes the public goods game, the bits layout, kernel AUTO, tile 0, "
                        "group 0 and the 16-colour schedule");
        return PGG_E_INVAL;
    }
    if (((uintptr_t)dev_lattice & 3u) != 0 || ((uintptr_t)dev_counts & 7u) != 0) {
        pgg::set_errorf("dev_lattice must be 4-byte and dev_counts 8-byte aligned");
        return PGG_E_INVAL;
    }
    if (t0 + (uint64_t)n_sweeps > 4294967296ull) { pgg::set_errorf("sweep index would exceed 2^32"); return PGG_E_INVAL; }
    if (n_sweeps == 0) return PGG_OK;

    hipStream_t st = (hipStream_t)hip_stream;
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    unsigned char* base = nullptr;
    if (e == hipSuccess) e = scratch_address(device, &base);
    if (e != hipSuccess) {
        pgg::set_errorf("pgg_sweep_static: scratch address: %s", hipGetErrorString(e));
        return PGG_E_DEVICE;
    }
    pgg::EnsRep* d_rep = (pgg::EnsRep*)(base + kOffRep);
    uint32_t* d_T = (uint32_t*)(base + kOffTable);
    unsigned long long* d_nc = (unsigned long long*)(base + kOffNc);
    unsigned long long* d_counts_own = (unsigned long long*)(base + kOffCounts);
    unsigned long long* d_delta = (unsigned long long*)(base + kOffDelta);
    uint32_t* d_lat2 = (uint32_t*)(base + kOffLat2);

    bool pair = false;
    int segw = 0;
    pgg::auto_segment_plan(p->L, device, &pair, &segw);
    pgg::EnsRep rp;
    std::memset(&rp, 0, sizeof(rp));
    pgg::ens_geometry(rp, (int)p->L, segw);
    rp.lat = (uint32_t*)dev_lattice;
    rp.lat2 = d_lat2;
    rp.T = d_T;
    rp.delta = d_delta;
    rp.nc = d_nc;
    rp.drawn = nullptr;
    rp.k0 = (uint32_t)p->seed;
    rp.k1 = (uint32_t)(p->seed >> 32);
    rp.t0 = (uint32_t)t0;
    TableArg tab;
    pgg::fermi_table(p->r, p->K, tab.T);

    hipLaunchKernelGGL(k_static_setup, dim3(1), dim3(256), 0, st, d_rep, rp, d_T, tab);
    e = hipGetLastError();
    // N_C(t0) of the caller's lattice: the base of the per-sweep counts
    if (e == hipSuccess) e = pgg::launch_count(PGG_LAYOUT_BITS, dev_lattice, (int)p->L, rp.stride, d_nc, st);
    const int blocks = pair ? pgg::pair_blocks(rp) : pgg::ens_waves(rp);
    const size_t lds = pair ? pgg::pair_lds_bytes(rp.segw) : pgg::ens_lds_bytes(pgg::ens_wave_words(rp));
    uint32_t done = 0;
    while (e == hipSuccess && done < n_sweeps) {
        const int len = (int)std::min<uint32_t>((uint32_t)kStaticChunk, n_sweeps - done);
        unsigned long long* counts = dev_counts ? (unsigned long long*)dev_counts + done : d_counts_own;
        e = pair ? pgg::launch_pair_chunk(d_rep, blocks, lds, len, kStaticChunk, counts, st, nullptr)
                 : pgg::launch_ens_chunk(d_rep, 1, blocks, lds, len, kStaticChunk, true, counts, st);
        done += (uint32_t)len;
    }
    if (e != hipSuccess) {
        pgg::set_errorf("pgg_sweep_static: launch failed: %s", hipGetErrorString(e));
        return PGG_E_DEVICE;
    }
    return PGG_OK;
}

}  // extern "C"
