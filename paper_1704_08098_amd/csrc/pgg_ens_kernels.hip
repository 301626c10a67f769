// Device side of the batched ensemble: the per-residue segment and paired
// kernels over the replica table, the chunk bookkeeping kernels (counter
// zeroing, count scan, sweep-index advance, copy-back of odd chunks) and
// their launchers.  The host engine that owns the replicas, captures the
// chunk graphs and tunes them is pgg_ensemble.hip.
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
        // Wave wid stages window rows wid, wid + NW, ..; lane l words l and
        // l + 64 of each (128 words per pass).  Every load of a pass is
        // issued before the first LDS store, so a wave waits for one round
        // trip to L2 per pass, not one per word.
        constexpr int NR = (B + 12 + NW - 1) / NW;  // window rows per wave
        const int w0 = c0 >> 5;  // segments start on word boundaries (L % 32 == 0)
        for (int wb = 0; wb < WB; wb += 128) {
            int widx[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                int x = w0 + wb + 64 * u + lane;  // in [-2, nw + 2) where the word is staged
                x += (x < 0) ? nw : 0;
                x -= (x >= nw) ? nw : 0;
                widx[u] = x;
            }
            uint32_t v[2][NR];
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const int o = wid + NW * j;
                int gi = R0 - 6 + o;  // in [-6, L + B + 6)
                gi += (gi < 0) ? L : 0;
                gi -= (gi >= L) ? L : 0;
                const uint32_t* src = (((gi & 3) < a) ? next : cur) + (size_t)gi * stride;
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int w = wb + 64 * u + lane;
                    v[u][j] = (o < B + 12 && w < WB) ? src[widx[u]] : 0u;
                }
            }
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const int o = wid + NW * j;
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int w = wb + 64 * u + lane;
                    if (o < B + 12 && w < WB) wwin[o * WB + w] = v[u][j];
                }
            }
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
    // the tiled schedule and the resident kernel update in place
    if (rp.tiled || rp.resident || (rp.n_active & 1) == 0) return;
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
    if (lds > 64 * 1024) {  // wide explicit tiles: the per-kernel LDS attribute
        const void* kern = wpg == 2 ? (const void*)k_ens_segment<2>
                                    : wpg == 4 ? (const void*)k_ens_segment<4> : (const void*)k_ens_segment<8>;
        if (!allow_dynamic_lds(kern, lds)) return hipErrorInvalidValue;
    }
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

hipError_t launch_pair_chunk(EnsRep* d_rep, int blocks, size_t lds, int len, int chunk, unsigned long long* counts,
                             hipStream_t st, unsigned long long* span) {
    if (!allow_dynamic_lds((const void*)k_ens_pair<kPairBand>, lds)) return hipErrorInvalidValue;
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

