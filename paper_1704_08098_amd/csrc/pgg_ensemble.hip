// Batched ensemble: many independent lattices (replicas of uneven L, r and
// seed) advanced together.  Every launch covers one row residue of one sweep
// of every replica: the waves of the launch are dealt out replica by replica
// (each replica's waves padded to whole workgroups, so a workgroup serves one
// replica and shares its threshold table), and each wave runs the segment
// update of one row segment.  A chunk of sweeps -- zeroing the per-sweep
// counters, 4 launches per sweep, the per-replica count scan and the advance
// of every replica's sweep index -- is captured once in a hipGraph and
// replayed; the sweep index lives in device memory so the same graph serves
// every chunk.  Results are those of the replicas run one by one.
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
#include "pgg_fullrow.hpp"
#include "pgg_segment.hpp"

namespace pgg {

// Replica whose wave range holds wave w: the last replica with wave_base <= w.
__device__ __forceinline__ int replica_of_wave(const EnsRep* __restrict__ reps, int n, int w) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (reps[mid].wave_base <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int WPG>
__global__ void __launch_bounds__(64 * WPG)
k_ens_segment(const EnsRep* __restrict__ reps, int n_reps, int a, int q, unsigned long long* __restrict__ span) {
    extern __shared__ uint32_t smem[];
    __shared__ int s_part[2 * WPG];
    const unsigned long long t_begin = span ? wall_clock64() : 0ull;
    const int lane = threadIdx.x & 63;
    // Everything below that depends only on the wave (its replica, row and
    // segment) is wave-uniform: readfirstlane keeps it in scalar registers.
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // neighbouring rows (which share window rows) run on the same XCD's L2
    const int first_wave = xcd_major((int)blockIdx.x, (int)gridDim.x) * WPG;
    const int rep_id = __builtin_amdgcn_readfirstlane(replica_of_wave(reps, n_reps, first_wave));
    const EnsRep rp = reps[rep_id];
    uint32_t* sT = smem;
    uint32_t* win = smem + kSegTableWords + wid * rep_wave_words(rp);
    const int lw = first_wave + wid - rp.wave_base;  // wave index inside the replica
    // sweep q of the chunk reads the state after sweep q - 1: lat for even q,
    // lat2 for odd q, and writes the other buffer.
    const uint32_t* cur = (q & 1) ? rp.lat2 : rp.lat;
    uint32_t* next = (q & 1) ? rp.lat : rp.lat2;
    const uint32_t t = rp.t0 + (uint32_t)q;
    int my_delta = 0, my_drawn = 0;
    seg_load_table(sT, rp.T);
    if (rp.rpw > 0) {
        // whole rows: wave lw owns rows a + 4 (lw R + r), r < nrows
        const int R = rp.rpw, rows = rp.L >> 2;
        const bool active = q < rp.n_active && lw * R < rows;
        const int i0 = a + 4 * lw * R;
        const int nrows = min(R, rows - lw * R);
        if (active) fullrow_fill(cur, next, rp.L, rp.stride, a, i0, R, win);
        __syncthreads();
        if (active) fullrow_run(next, rp.L, rp.stride, a, i0, R, nrows, t, rp.k0, rp.k1, sT, win, my_delta, my_drawn);
    } else {
        const bool active = q < rp.n_active && lw < (rp.L >> 2) * rp.nseg;
        const SegPos g = seg_pos(rp.L, a, rp.segw, active ? lw / rp.nseg : 0, active ? lw % rp.nseg : 0);
        if (active) segment_fill(cur, next, rp.L, rp.stride, rp.nw, a, rp.segw, g, win);
        __syncthreads();
        if (active)
            segment_run(next, rp.L, rp.stride, a, rp.segw, g, t, rp.k0, rp.k1, sT, win, rp.drawn != nullptr, my_delta,
                        my_drawn);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        my_delta += __shfl_xor(my_delta, off, 64);
        my_drawn += __shfl_xor(my_drawn, off, 64);
    }
    if (lane == 0) {
        s_part[wid] = my_delta;
        s_part[WPG + wid] = my_drawn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int dsum = 0, nsum = 0;
        for (int k = 0; k < WPG; ++k) {
            dsum += s_part[k];
            nsum += s_part[WPG + k];
        }
        if (dsum)
            atomicAdd(slot_of(rp.delta + (size_t)q * kSweepWords, (int)blockIdx.x),
                      (unsigned long long)(long long)dsum);
        if (rp.drawn && nsum) atomicAdd(slot_of(rp.drawn, (int)blockIdx.x), (unsigned long long)nsum);
        if (span) {  // diagnostics: earliest start and latest end over kSpanSlots spread pairs
            unsigned long long* sp = span + 2 * (blockIdx.x & (kSpanSlots - 1));
            atomicMin(sp, t_begin);
            atomicMax(sp + 1, wall_clock64());
        }
    }
}

// Two row residues per launch (residues a and a + 1, a = 0 or 2) for one
// lattice (reps[0], segments of rp.segw columns, L a multiple of 32).  A
// workgroup stages rows R0 - 6 .. R1 + 5 of its band [R0, R1) (kPairBand rows)
// and its segment's columns s - 64 .. e + 63 once.  Residue a then runs on its
// rows in [R0 - 1, R1 + 3) -- those a row of residue a + 1 in the band reads
// (rows i - 1 and i + 3) -- each class with 12 more margin columns, so that
// every row and column the second residue reads is exact; after a workgroup
// barrier residue a + 1 runs on the band's rows.
// Only band rows and owned columns are written back and counted.  Rows of
// residue below a come from next (this sweep), the others from cur.
template <int B>
__global__ void __launch_bounds__(64 * (B / 4 + 1))
k_ens_pair(const EnsRep* __restrict__ reps, int a, int q, unsigned long long* __restrict__ span) {
    constexpr int NW = B / 4 + 1;
    extern __shared__ uint32_t smem[];
    __shared__ int s_part[2 * NW];
    const unsigned long long t_begin = span ? wall_clock64() : 0ull;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const EnsRep rp = reps[0];
    const int L = rp.L, segw = rp.segw, nseg = rp.nseg, stride = rp.stride, nw = rp.nw;
    const int WB = seg_window_words(segw), cap = seg_list_cap(segw);
    const int blk = xcd_major((int)blockIdx.x, (int)gridDim.x);  // neighbouring bands share an XCD
    const int band = blk / nseg, sg = blk - band * nseg;
    const int R0 = band * B, R1 = min(R0 + B, L);
    const int s = sg * segw, e = min(L, s + segw), c0 = s - 64;
    uint32_t* sT = smem;
    uint32_t* wwin = smem + kSegTableWords;  // (B + 12) rows x WB
    uint32_t* lists = wwin + (B + 12) * WB;  // NW x cap
    const bool on = q < rp.n_active;
    const uint32_t* cur = (q & 1) ? rp.lat2 : rp.lat;
    uint32_t* next = (q & 1) ? rp.lat : rp.lat2;
    const uint32_t t = rp.t0 + (uint32_t)q;
    seg_load_table(sT, rp.T);
    if (on) {
        const int w0 = c0 >> 5;  // segments start on word boundaries (L % 32 == 0)
        for (int k = threadIdx.x; k < (B + 12) * WB; k += blockDim.x) {
            const int o = k / WB, w = k - o * WB;
            int gi = R0 - 6 + o;  // in [-6, L + B + 6)
            gi += (gi < 0) ? L : 0;
            gi -= (gi >= L) ? L : 0;
            int widx = w0 + w;  // in [-2, nw + 2)
            widx += (widx < 0) ? nw : 0;
            widx -= (widx >= nw) ? nw : 0;
            const uint32_t* src = ((gi & 3) < a) ? next : cur;
            wwin[k] = src[(size_t)gi * stride + widx];
        }
    }
    __syncthreads();
    int my_delta = 0, my_drawn = 0;
    // residue a: rows in [R0 - 1, R1 + 3) (R0 is a multiple of 4)
    {
        const int i = R0 - 1 + ((a + 1) & 3) + 4 * wid;
        if (on && i < R1 + 3) {
            const int gi = i < 0 ? i + L : (i >= L ? i - L : i);
            const SegPos g = {gi, s, e, c0};
            segment_run_row(next, L, stride, a, segw, g, t, rp.k0, rp.k1, sT, wwin + (i - (R0 - 6)) * WB,
                            lists + wid * cap, 12, i >= R0 && i < R1, rp.drawn != nullptr, my_delta, my_drawn);
        }
    }
    __syncthreads();
    // residue a + 1: band rows (R0 is a multiple of 4)
    {
        const int i = R0 + a + 1 + 4 * wid;
        if (on && i < R1) {
            const SegPos g = {i, s, e, c0};
            segment_run_row(next, L, stride, a + 1, segw, g, t, rp.k0, rp.k1, sT, wwin + (i - (R0 - 6)) * WB,
                            lists + wid * cap, 0, true, rp.drawn != nullptr, my_delta, my_drawn);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        my_delta += __shfl_xor(my_delta, off, 64);
        my_drawn += __shfl_xor(my_drawn, off, 64);
    }
    if (lane == 0) {
        s_part[wid] = my_delta;
        s_part[NW + wid] = my_drawn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int dsum = 0, nsum = 0;
        for (int k = 0; k < NW; ++k) {
            dsum += s_part[k];
            nsum += s_part[NW + k];
        }
        if (dsum)
            atomicAdd(slot_of(rp.delta + (size_t)q * kSweepWords, (int)blockIdx.x),
                      (unsigned long long)(long long)dsum);
        if (rp.drawn && nsum) atomicAdd(slot_of(rp.drawn, (int)blockIdx.x), (unsigned long long)nsum);
        if (span) {
            unsigned long long* sp = span + 2 * (blockIdx.x & (kSpanSlots - 1));
            atomicMin(sp, t_begin);
            atomicMax(sp + 1, wall_clock64());
        }
    }
}

// Per replica: counts[rep][q] = nc[rep] + prefix over q of the sweep deltas
// (q < n_active), then nc[rep] advances.  One block per replica.
__global__ void __launch_bounds__(256)
k_ens_scan(const EnsRep* __restrict__ reps, int K, unsigned long long* __restrict__ counts) {
    __shared__ unsigned long long part[256];
    const EnsRep& rp = reps[blockIdx.x];
    const int n = min(rp.n_active, K);
    const int tid = threadIdx.x;
    const int chunk = (n + 255) / 256;
    const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
    auto sweep_delta = [&](int q) {
        unsigned long long v = 0;
        const unsigned long long* row = rp.delta + (size_t)q * kSweepWords;
        for (int k = 0; k < kSlots; ++k) v += row[k * kSlotStride];
        return v;
    };
    unsigned long long sum = 0;
    for (int q = lo; q < hi; ++q) sum += sweep_delta(q);
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const unsigned long long v = tid >= off ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    unsigned long long run = *rp.nc + (tid ? part[tid - 1] : 0ull);
    for (int q = lo; q < hi; ++q) {
        run += sweep_delta(q);
        counts[(size_t)blockIdx.x * K + q] = run;
    }
    __syncthreads();
    if (tid == 255) *rp.nc += part[255];
}

// After a chunk whose replica ran an odd number of sweeps, its state is in
// lat2: copy it back (blockIdx.x = replica, kCopyBlocks blocks per replica
// share its words).
constexpr int kCopyBlocks = 64;
__global__ void k_ens_copyback(const EnsRep* __restrict__ reps) {
    const EnsRep& rp = reps[blockIdx.x];
    if (rp.tiled || (rp.n_active & 1) == 0) return;  // the tiled schedule updates in place
    const int n = rp.L * rp.stride;
    for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < n; k += gridDim.y * blockDim.x) rp.lat[k] = rp.lat2[k];
}

// Zero the per-sweep counters of every replica (one block per replica).
__global__ void k_ens_zero(const EnsRep* __restrict__ reps, int chunk) {
    unsigned long long* d = reps[blockIdx.x].delta;
    const int n = chunk * kSlots;  // only the slot words of each sweep's row are used
    for (int k = threadIdx.x; k < n; k += blockDim.x) d[(size_t)(k / kSlots) * kSweepWords + (k % kSlots) * kSlotStride] = 0ull;
}

// Sweep bookkeeping of every replica: n_active for the next chunk, or the
// advance of t0 after it.
__global__ void k_ens_set_active(EnsRep* __restrict__ reps, int n_reps, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_reps) reps[k].n_active = n;
}

__global__ void k_ens_advance(EnsRep* __restrict__ reps, int n_reps) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_reps) reps[k].t0 += (uint32_t)reps[k].n_active;
}

__global__ void k_ens_set_t0(EnsRep* __restrict__ reps, int n_reps, uint32_t t0) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_reps) reps[k].t0 = t0;
}

__global__ void k_span_reset(unsigned long long* span, int n_words) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_words) span[k] = (k & 1) ? 0ull : ~0ull;
}

hipError_t launch_span_reset(unsigned long long* span, int n_launches, hipStream_t st) {
    const int n = kSpanWords * n_launches;
    hipLaunchKernelGGL(k_span_reset, dim3((n + 255) / 256), dim3(256), 0, st, span, n);
    return hipGetLastError();
}

hipError_t launch_ens_set_t0(EnsRep* d_reps, int n, uint32_t t0, hipStream_t st) {
    hipLaunchKernelGGL(k_ens_set_t0, dim3((n + 255) / 256), dim3(256), 0, st, d_reps, n, t0);
    return hipGetLastError();
}

int auto_segw(int L) {
    if (L % 32 == 0 && L <= 1024) return L;  // whole rows
    // About 1376 columns: at the drawn fraction of a lattice near r_c (about
    // 15 % of the sites) a class then lists about 50 sites, most of one
    // 64-lane pass; the row is split into equal segments of that order.  A
    // segment is at most L - 32 columns, so a row always takes two or more:
    // split it evenly (one segment of L - 32 columns and one of the rest
    // would leave the second wave almost empty).
    const int nseg = std::max(2, (L + 1375) / 1376);
    int w = (L / nseg + 31) & ~31;
    const int cap = (L - 32) & ~31;
    if (w > cap) w = cap;
    if (w < 32) w = 32;
    return w;
}

bool segw_valid(int L, int segw) {
    if (segw == L) return L % 32 == 0;
    return segw > 0 && segw % 32 == 0 && segw + 32 <= L;
}

void ens_geometry(EnsRep& rp, int L, int segw) {
    if (segw == 0) segw = auto_segw(L);
    rp.L = L;
    rp.stride = 2 * ((L + 63) / 64);
    rp.nw = (L + 31) / 32;
    rp.segw = segw;
    if (segw == L) {
        rp.nseg = 1;
        const int R = L >= 1024 ? 1 : 1024 / L;
        rp.rpw = R < L / 4 ? R : L / 4;
    } else {
        rp.nseg = (L + segw - 1) / segw;
        rp.rpw = 0;
    }
}

int ens_waves(const EnsRep& rp, int wpg) {
    const int rows = rp.L / 4;
    const int wv = rp.rpw > 0 ? (rows + rp.rpw - 1) / rp.rpw : rows * rp.nseg;
    return (wv + wpg - 1) / wpg * wpg;
}

int ens_wave_words(const EnsRep& rp) { return rep_wave_words(rp); }

size_t ens_lds_bytes(int max_wave_words, int wpg) {
    return (kSegTableWords + (size_t)wpg * max_wave_words) * sizeof(uint32_t);
}

bool ens_wpg_valid(int wpg) { return wpg == 2 || wpg == 4 || wpg == 8; }

hipError_t launch_ens_begin(EnsRep* d_reps, int n, int len, int chunk, bool set_active, hipStream_t st) {
    if (set_active) {
        hipLaunchKernelGGL(k_ens_set_active, dim3((n + 255) / 256), dim3(256), 0, st, d_reps, n, len);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(k_ens_zero, dim3(n), dim3(256), 0, st, d_reps, chunk);
    return hipGetLastError();
}

hipError_t launch_ens_residue(const EnsRep* d_reps, int n, int total_waves, size_t lds, int a, int q,
                              hipStream_t st, int wpg, unsigned long long* span) {
    const dim3 grid(total_waves / wpg), block(64 * wpg);
    switch (wpg) {
        case 2: hipLaunchKernelGGL(k_ens_segment<2>, grid, block, lds, st, d_reps, n, a, q, span); break;
        case 4: hipLaunchKernelGGL(k_ens_segment<4>, grid, block, lds, st, d_reps, n, a, q, span); break;
        case 8: hipLaunchKernelGGL(k_ens_segment<8>, grid, block, lds, st, d_reps, n, a, q, span); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ens_end(EnsRep* d_reps, int n, int chunk, unsigned long long* counts, hipStream_t st) {
    hipError_t err;
    hipLaunchKernelGGL(k_ens_scan, dim3(n), dim3(256), 0, st, d_reps, chunk, counts);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(k_ens_copyback, dim3(n, kCopyBlocks), dim3(256), 0, st, d_reps);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(k_ens_advance, dim3((n + 255) / 256), dim3(256), 0, st, d_reps, n);
    return hipGetLastError();
}

hipError_t launch_ens_chunk(EnsRep* d_reps, int n, int total_waves, size_t lds, int len, int chunk,
                            bool set_active, unsigned long long* counts, hipStream_t st, int wpg,
                            unsigned long long* span) {
    hipError_t err = launch_ens_begin(d_reps, n, len, chunk, set_active, st);
    for (int q = 0; err == hipSuccess && q < len; ++q)
        for (int a = 0; err == hipSuccess && a < 4; ++a)
            err = launch_ens_residue(d_reps, n, total_waves, lds, a, q, st, wpg,
                                     span ? span + kSpanWords * (4 * q + a) : nullptr);
    if (err != hipSuccess) return err;
    return launch_ens_end(d_reps, n, chunk, counts, st);
}

size_t pair_lds_bytes(int segw) {
    return (kSegTableWords + (size_t)(kPairBand + 12) * seg_window_words(segw) +
            (size_t)(kPairBand / 4 + 1) * seg_list_cap(segw)) * sizeof(uint32_t);
}

int pair_blocks(const EnsRep& rp) { return (rp.L + kPairBand - 1) / kPairBand * rp.nseg; }

hipError_t launch_pair_chunk(EnsRep* d_rep, int blocks, size_t lds, int len, int chunk, unsigned long long* counts,
                             hipStream_t st, unsigned long long* span) {
    hipError_t err = launch_ens_begin(d_rep, 1, len, chunk, true, st);
    for (int q = 0; err == hipSuccess && q < len; ++q)
        for (int h = 0; err == hipSuccess && h < 2; ++h) {
            hipLaunchKernelGGL(k_ens_pair<kPairBand>, dim3(blocks), dim3(64 * (kPairBand / 4 + 1)), lds, st, d_rep,
                               2 * h, q, span ? span + kSpanWords * (2 * q + h) : nullptr);
            err = hipGetLastError();
        }
    if (err != hipSuccess) return err;
    return launch_ens_end(d_rep, 1, chunk, counts, st);
}

}  // namespace pgg

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
    if (e->d_lattices) (void)hipFree(e->d_lattices);
    if (e->d_tables) (void)hipFree(e->d_tables);
    if (e->d_delta) (void)hipFree(e->d_delta);
    if (e->d_counts) (void)hipFree(e->d_counts);
    if (e->d_nc) (void)hipFree(e->d_nc);
    if (e->capture_stream) (void)hipStreamDestroy(e->capture_stream);
    for (hipStream_t bs : e->branch_streams) (void)hipStreamDestroy(bs);
    for (hipEvent_t ev : e->branch_events) (void)hipEventDestroy(ev);
    if (e->own_stream && e->stream) (void)hipStreamDestroy(e->stream);
    delete e;
}

hipError_t enqueue_chunk(pgg_ensemble* e, int len, hipStream_t st) {
    if (e->tiled)
        return pgg::launch_ens_tiled_chunk(e->d_reps, e->n, e->total_waves, len, e->chunk, e->d_counts, st);
    if (e->branches == 1)
        return pgg::launch_ens_chunk(e->d_reps, e->n, e->total_waves, e->lds, len, e->chunk, true, e->d_counts, st,
                                     e->wpg);
    // fork: every branch waits for the work before it on st, runs its range's
    // chunk, and st waits for every branch (a graph with parallel branches)
    hipError_t err = hipEventRecord(e->branch_events[0], st);
    for (int g = 0; err == hipSuccess && g < e->branches; ++g) {
        hipStream_t bs = e->branch_streams[g];
        err = hipStreamWaitEvent(bs, e->branch_events[0], 0);
        if (err == hipSuccess)
            err = pgg::launch_ens_chunk(e->d_reps + e->grp_first[g], e->grp_count[g], e->grp_waves[g], e->lds, len,
                                        e->chunk, true, e->d_counts + (size_t)e->grp_first[g] * e->chunk, bs, e->wpg);
        if (err == hipSuccess) err = hipEventRecord(e->branch_events[1 + g], bs);
        if (err == hipSuccess) err = hipStreamWaitEvent(st, e->branch_events[1 + g], 0);
    }
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
            eerr("replica %u: the tiled schedule needs L % 8 == 0 and tile 0", k);
            return PGG_E_INVAL;
        }
        const uint32_t w = tiles ? tiles[k] : 0;
        if (w != 0 && !pgg::segw_valid((int)p.L, (int)w)) { eerr("replica %u: tile must be a multiple of 32 and <= L - 32, or L (whole rows, L a multiple of 32)", k); return PGG_E_INVAL; }
    }
    return PGG_OK;
}

}  // namespace

extern "C" {

pgg_status pgg_ensemble_create(const pgg_params* reps, uint32_t n_reps, const uint32_t* tiles, uint32_t chunk,
                               uint32_t waves_per_group, uint32_t branches, void* hip_stream, pgg_ensemble** out) {
    if (!out) { eerr("out is NULL"); return PGG_E_INVAL; }
    *out = nullptr;
    const pgg_status vs = validate_reps(reps, n_reps, tiles, chunk);
    if (vs != PGG_OK) return vs;
    const int wpg = waves_per_group ? (int)waves_per_group : pgg::kWavesPerGroup;
    if (!pgg::ens_wpg_valid(wpg)) { eerr("waves_per_group must be 0, 2, 4 or 8"); return PGG_E_INVAL; }
    if (branches > 16) { eerr("branches must lie in [0, 16]"); return PGG_E_INVAL; }
    if (branches > 1 && reps[0].schedule == PGG_SCHEDULE_TILED) { eerr("the tiled schedule runs one branch"); return PGG_E_INVAL; }
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
    e->tiled = reps[0].schedule == PGG_SCHEDULE_TILED;
    if (hipGetDevice(&e->device) != hipSuccess) { eerr("no HIP device"); ens_release(e); return PGG_E_DEVICE; }

    // Layout: lattices back to back (256-byte aligned), tables, per-replica waves.
    std::vector<size_t> lat_off(n_reps);
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
        waves += e->tiled ? pgg::tiled_blocks(rp.L) : pgg::ens_waves(rp, wpg);
        lat_off[k] = lat_words;
        lat_words += (e->tiled ? 1 : 2) * (((size_t)rp.L * rp.stride + 63) & ~(size_t)63);  // lat (and lat2)
        if (!e->tiled) max_words = std::max(max_words, pgg::ens_wave_words(rp));
    }
    e->total_waves = waves;
    e->lds = e->tiled ? 0 : pgg::ens_lds_bytes(max_words, wpg);
    // contiguous replica ranges of about equal work; wave_base restarts in each
    e->branches = std::max(1, std::min<int>(branches ? (int)branches : 1, (int)n_reps));
    {
        double total_work = 0.0;
        for (uint32_t k = 0; k < n_reps; ++k) total_work += (double)reps[k].L * (double)reps[k].L;
        double acc = 0.0;
        int g = 0, base = 0;
        e->grp_first.assign(1, 0);
        for (uint32_t k = 0; k < n_reps; ++k) {
            pgg::EnsRep& rp = e->host_reps[k];
            // start the next range once this one holds its share of the work
            // (every range keeps at least one replica)
            if (g + 1 < e->branches && k > (uint32_t)e->grp_first[g] &&
                acc >= total_work * (double)(g + 1) / (double)e->branches) {
                e->grp_waves.push_back(base);
                e->grp_count.push_back((int)k - e->grp_first[g]);
                e->grp_first.push_back((int)k);
                ++g;
                base = 0;
            }
            rp.wave_base = base;
            if (!e->tiled) base += pgg::ens_waves(rp, wpg);
            acc += (double)reps[k].L * (double)reps[k].L;
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
    for (int g = 0; e->branches > 1 && g < e->branches; ++g) {
        hipStream_t bs = nullptr;
        if (hipStreamCreateWithFlags(&bs, hipStreamNonBlocking) != hipSuccess) { eerr("stream creation failed"); ens_release(e); return PGG_E_DEVICE; }
        e->branch_streams.push_back(bs);
    }
    for (int g = 0; e->branches > 1 && g <= e->branches; ++g) {
        hipEvent_t ev = nullptr;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) { eerr("event creation failed"); ens_release(e); return PGG_E_DEVICE; }
        e->branch_events.push_back(ev);
    }
    if (e->lds > pgg::kMaxDynamicLds) {
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
                                 uint32_t* tiles_out, uint32_t* chunk_out, uint32_t* wpg_out, uint32_t* branches_out,
                                 double* ms_out) {
    if (!reps || !tiles_out || !chunk_out || !wpg_out || !branches_out) { eerr("NULL argument"); return PGG_E_INVAL; }
    if (probe_sweeps == 0 || probe_sweeps > 4096) { eerr("probe_sweeps must lie in [1, 4096]"); return PGG_E_INVAL; }
    const pgg_status vs = validate_reps(reps, n_reps, nullptr, 1);
    if (vs != PGG_OK) return vs;
    if (reps[0].schedule == PGG_SCHEDULE_TILED) { eerr("the tiled schedule has nothing to tune"); return PGG_E_INVAL; }
    std::vector<uint32_t> sizes;
    for (uint32_t k = 0; k < n_reps; ++k)
        if (std::find(sizes.begin(), sizes.end(), reps[k].L) == sizes.end()) sizes.push_back(reps[k].L);
    std::map<uint32_t, uint32_t> width;  // current choice per L (0 = automatic)
    for (uint32_t L : sizes) width[L] = 0;
    uint32_t chunk = 32, wpg = (uint32_t)pgg::kWavesPerGroup, branches = 1;
    std::vector<uint64_t> fingerprint, nc(n_reps);
    std::vector<uint32_t> tiles(n_reps);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess) {
        if (ev0) (void)hipEventDestroy(ev0);
        eerr("event creation failed");
        return PGG_E_DEVICE;
    }
    // One trial: a fresh ensemble with the current choices; best of two timed runs.
    auto trial = [&](double* ms) -> pgg_status {
        for (uint32_t k = 0; k < n_reps; ++k) tiles[k] = width[reps[k].L];
        pgg_ensemble* e = nullptr;
        pgg_status st = pgg_ensemble_create(reps, n_reps, tiles.data(), chunk, wpg, branches, hip_stream, &e);
        if (st != PGG_OK) return st;
        st = pgg_ensemble_sweep(e, 2, nullptr);
        double best = 1e300;
        for (int rep = 0; rep < 2 && st == PGG_OK; ++rep) {
            hipError_t err = hipEventRecord(ev0, e->stream);
            if (err == hipSuccess) st = pgg_ensemble_sweep(e, probe_sweeps, nullptr);
            if (err == hipSuccess && st == PGG_OK) err = hipEventRecord(ev1, e->stream);
            if (err == hipSuccess && st == PGG_OK) err = hipEventSynchronize(ev1);
            float f = 0.f;
            if (err == hipSuccess && st == PGG_OK) err = hipEventElapsedTime(&f, ev0, ev1);
            if (err != hipSuccess) { eerr("autotune timing: %s", hipGetErrorString(err)); st = PGG_E_DEVICE; }
            best = std::min(best, (double)f / probe_sweeps);
        }
        if (st == PGG_OK) st = pgg_ensemble_coop_counts(e, nc.data());
        pgg_ensemble_destroy(e);
        if (st != PGG_OK) return st;
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
    pgg_status st = trial(&best_ms);
    for (size_t q = 0; q < sizes.size() && st == PGG_OK; ++q) {
        const uint32_t L = sizes[q];
        const uint32_t cap = (L - 32) & ~31u;
        std::vector<uint32_t> cand;
        for (uint32_t w = 64; w < cap; w *= 2) cand.push_back(w);
        if (cap >= 32) cand.push_back(cap);
        if (L % 32 == 0) cand.push_back(L);  // whole rows
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
    const uint32_t branch_counts[] = {1, 2, 4};
    uint32_t best_branches = branches;
    for (uint32_t bcount : branch_counts) {
        if (st != PGG_OK || bcount == best_branches || bcount > n_reps) continue;
        branches = bcount;
        double ms = 0.0;
        st = trial(&ms);
        if (st == PGG_OK && ms < best_ms) { best_ms = ms; best_branches = bcount; }
    }
    branches = best_branches;
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
    *chunk_out = best_chunk;
    *wpg_out = best_wpg;
    *branches_out = best_branches;
    if (ms_out) *ms_out = best_ms;
    return PGG_OK;
}

pgg_status pgg_ensemble_run(const pgg_params* reps, uint32_t n_reps, uint32_t n_sweeps, uint64_t* counts,
                            const pgg_ensemble_tune* tune, void* hip_stream) {
    const pgg_status vs = validate_reps(reps, n_reps, tune ? tune->tiles : nullptr, tune ? tune->chunk : 1);
    if (vs != PGG_OK) return vs;
    std::vector<uint32_t> tiles;
    uint32_t chunk = 32, wpg = 0, branches = 0;
    if (tune) {
        chunk = tune->chunk;
        wpg = tune->waves_per_group;
        branches = tune->branches;
        if (tune->tiles) tiles.assign(tune->tiles, tune->tiles + n_reps);
    } else if (reps[0].schedule != PGG_SCHEDULE_TILED) {
        tiles.resize(n_reps);
        const pgg_status st = pgg_ensemble_autotune(reps, n_reps, 8, hip_stream, tiles.data(), &chunk, &wpg,
                                                    &branches, nullptr);
        if (st != PGG_OK) return st;
    }
    pgg_ensemble* e = nullptr;
    pgg_status st = pgg_ensemble_create(reps, n_reps, tiles.empty() ? nullptr : tiles.data(), chunk, wpg, branches,
                                        hip_stream, &e);
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
