// Persistent strip kernel: every workgroup owns H consecutive rows of one
// lattice for a whole run of sweeps, keeps them (plus a 3-row halo above and
// below) in LDS, and exchanges only its 3 top and 3 bottom rows with the two
// workgroups that own the neighbouring strips.  gfx950.
//
// A sweep is four steps, one per row residue a = i mod 4; step a runs the
// colour classes k = 4a + 0..3 of the strip's rows with i mod 4 = a.  Those
// rows read rows i-3..i+3, which are never updated in the same step, so a
// step of one strip depends only on the previous step of its two neighbours.
// After every step a workgroup publishes its first and last 3 rows into a
// two-slot ring in global memory; before the next step it copies the
// neighbours' rows of the previous step into its halo.  No grid-wide barrier
// and no cache-wide fence: every 64-bit ring word carries 32 strategy bits
// and a 32-bit tag (the producer's step + 1), written and polled with relaxed
// device-scope atomics, so seeing the tag means seeing the data (the
// flag-per-word scheme of low-latency collectives).  Two slots suffice: a
// workgroup overwrites a slot only after it has read its neighbours' data of
// the step that needed the slot's previous contents.  Polling is bounded in
// time; a workgroup that gives up raises an abort flag that makes every
// other workgroup leave too.  All workgroups must be resident at once
// (cooperative launch).  A lattice held by one workgroup refreshes its halo
// from its own rows.
//
// Inside a step the work follows the staged scheme: the sites that can change
// in the four classes (a superset computed from the step-start state, see
// pgg_staged.hip) are listed, their Philox blocks drawn in one batch, then
// the classes are updated in order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pgg_device.hpp"
#include "pgg_internal.hpp"

namespace pgg {

namespace {

__device__ __forceinline__ uint64_t ring_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void ring_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t flag_load(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void flag_store(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

__global__ void __launch_bounds__(kStripThreads)
k_strip(const StripTask* __restrict__ tasks, int n_tasks, uint64_t* __restrict__ ring_base,
        uint32_t* __restrict__ abort_flag, uint64_t wait_ticks, int G) {
    extern __shared__ uint32_t smem[];
    __shared__ int s_count[4];
    __shared__ int s_delta;
    __shared__ int s_ok;

    const int me = xcd_major((int)blockIdx.x, n_tasks);  // neighbouring strips share an XCD
    const StripTask tk = tasks[me];
    const int L = tk.L, nw = tk.nw, ldw = nw + 1, H = tk.H, r0 = tk.r0, q4 = L >> 2;
    const int GQ = G * q4;  // list capacity per class
    const int tid = threadIdx.x;
    const bool single = tk.up == me;  // the strip is the whole lattice

    uint32_t* sT = smem;
    uint32_t* img = sT + 160;                 // H + 6 rows: global row r0 - 3 + rho
    uint32_t* actrow = img + (H + 6) * ldw;   // G rows
    uint32_t* c0row = actrow + G * ldw;       // G rows
    uint32_t* ent = c0row + G * ldw;          // 4 * GQ
    uint32_t* uw = ent + 4 * GQ;              // 4 * GQ
    const int ringw = 6 * nw;                 // 64-bit words per ring slot
    uint64_t* my_ring = ring_base + (size_t)me * 2 * ringw;

    for (int q = tid; q < kTableSize; q += blockDim.x) sT[q] = tk.T[q];
    for (int q = tid; q < (H + 6) * ldw; q += blockDim.x) {
        const int rho = q / ldw, w = q - (q / ldw) * ldw;
        int gi = r0 - 3 + rho;
        while (gi < 0) gi += L;
        while (gi >= L) gi -= L;
        img[q] = (w < nw) ? tk.lat[(size_t)gi * tk.stride + w] : 0u;
    }
    if (tid < 4) s_count[tid] = 0;
    if (tid == 0) s_delta = 0;
    __syncthreads();

    const int steps = 4 * tk.n;
    for (int s = 0; s < steps; ++s) {
        const int a = s & 3;
        const uint32_t t = tk.t0 + (uint32_t)(s >> 2);

        // ---- halo for this step -------------------------------------------
        if (s > 0) {
            if (single) {
                for (int q = tid; q < 3 * ldw; q += blockDim.x) {
                    img[q] = img[H * ldw + q];                      // rows r0-3..r0-1 = last 3
                    img[(H + 3) * ldw + q] = img[3 * ldw + q];      // rows r0+H..+2 = first 3
                }
            } else {
                // Copy the neighbours' boundary rows of step s - 1, waiting for
                // each word's tag.
                const int slot = (s - 1) & 1;
                const uint64_t* up_ring = ring_base + (size_t)tk.up * 2 * ringw + slot * ringw;
                const uint64_t* dn_ring = ring_base + (size_t)tk.down * 2 * ringw + slot * ringw;
                if (tid == 0) s_ok = 1;
                __syncthreads();
                int ok = 1;
                const uint64_t start = wall_clock64();
                for (int q = tid; q < 6 * nw && ok; q += blockDim.x) {
                    const int rr = q / nw, w = q - (q / nw) * nw;
                    // rows 0..2: up's last 3 rows (its ring rows 3..5) -> halo rows 0..2
                    // rows 3..5: down's first 3 rows (its ring rows 0..2) -> halo rows H+3..H+5
                    const uint64_t* src = rr < 3 ? up_ring + (3 + rr) * nw + w : dn_ring + (rr - 3) * nw + w;
                    uint64_t v = ring_load(src);
                    while ((uint32_t)(v >> 32) != (uint32_t)s) {
                        if (flag_load(abort_flag) != 0u) { ok = 0; break; }
                        if (wall_clock64() - start > wait_ticks) {
                            flag_store(abort_flag, 1u);
                            ok = 0;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                        v = ring_load(src);
                    }
                    img[(rr < 3 ? rr : H + rr) * ldw + w] = (uint32_t)v;
                }
                if (!ok) s_ok = 0;
                __syncthreads();
                if (!s_ok) return;  // every thread of the workgroup leaves here
            }
            __syncthreads();
        }

        // ---- the step: rows i = a mod 4 of the strip, in groups of G rows ----
        const int fa = r0 + ((a - (r0 & 3)) & 3);  // first strip row with i mod 4 = a
        const int Ra = fa < r0 + H ? (r0 + H - 1 - fa) / 4 + 1 : 0;
        for (int gbase = 0; gbase < Ra; gbase += G) {
            const int Gv = min(G, Ra - gbase);
            // A1: step-start activity and class-0 candidates
            for (int q = tid; q < Gv * ldw; q += blockDim.x) {
                const int m = q / ldw, w = q - (q / ldw) * ldw;
                uint32_t act = 0;
                if (w < nw) {
                    const uint32_t* rr = img + (fa + 4 * (gbase + m) - r0 + 3) * ldw;
                    const uint32_t X = rr[w];
                    const uint32_t E = row_window(rr, L, 32 * w + 1);
                    const uint32_t Wn = row_window(rr, L, 32 * w - 1);
                    const int valid = L - 32 * w;
                    const uint32_t vmask = valid >= 32 ? 0xFFFFFFFFu : ((1u << valid) - 1u);
                    act = ((X ^ E) | (X ^ Wn) | (X ^ rr[w - ldw]) | (X ^ rr[w + ldw])) & vmask;
                }
                actrow[q] = act;
                c0row[q] = act & 0x11111111u;
            }
            __syncthreads();
            // A2: classes 1..3 and the lists
            for (int q = tid; q < Gv * nw; q += blockDim.x) {
                const int m = q / nw, w = q - (q / nw) * nw;
                const uint32_t act = actrow[m * ldw + w];
                const uint32_t c0 = c0row[m * ldw + w];
                const int valid = L - 32 * w;
                const uint32_t vmask = valid >= 32 ? 0xFFFFFFFFu : ((1u << valid) - 1u);
                const uint32_t c1 = (act | (c0 << 1)) & 0x22222222u;
                const uint32_t c2 = (act | (c1 << 1)) & 0x44444444u;
                const uint32_t e0 = row_window(c0row + m * ldw, L, 32 * w + 1) & vmask;
                const uint32_t c3 = (act | (c2 << 1) | e0) & 0x88888888u;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    uint32_t bits = b == 0 ? c0 : b == 1 ? c1 : b == 2 ? c2 : c3;
                    const int cnt = __popc(bits);
                    if (cnt) {
                        int pos = atomicAdd(&s_count[b], cnt);
                        uint32_t* dst = ent + b * GQ;
                        while (bits) {
                            const int bit = __ffs(bits) - 1;
                            bits &= bits - 1u;
                            dst[pos++] = ((uint32_t)m << 16) | (uint32_t)(32 * w + bit);
                        }
                    }
                }
            }
            __syncthreads();
            // A3: Philox blocks of all candidates, two per lane per iteration
            const int n0 = s_count[0], n1 = s_count[1], n2 = s_count[2], n3 = s_count[3];
            const int total = n0 + n1 + n2 + n3;
            const uint32_t kbase = (uint32_t)(4 * a);
            const int rowbase = fa + 4 * gbase;
            for (int f = tid; f < total; f += 2 * (int)blockDim.x) {
                const int f2 = f + (int)blockDim.x;
                const bool two = f2 < total;
                const int fb = two ? f2 : f;
                const int b1 = (f >= n0) + (f >= n0 + n1) + (f >= n0 + n1 + n2);
                const int b2 = (fb >= n0) + (fb >= n0 + n1) + (fb >= n0 + n1 + n2);
                const int o1 = b1 == 0 ? 0 : b1 == 1 ? n0 : b1 == 2 ? n0 + n1 : n0 + n1 + n2;
                const int o2 = b2 == 0 ? 0 : b2 == 1 ? n0 : b2 == 2 ? n0 + n1 : n0 + n1 + n2;
                const int s1 = b1 * GQ + (f - o1), s2 = b2 * GQ + (fb - o2);
                const uint32_t e1 = ent[s1], e2 = ent[s2];
                const uint32_t x1 = (uint32_t)(rowbase + 4 * (int)(e1 >> 16)) * (uint32_t)L + (e1 & 0xFFFFu);
                const uint32_t x2 = (uint32_t)(rowbase + 4 * (int)(e2 >> 16)) * (uint32_t)L + (e2 & 0xFFFFu);
                const uint4 p1 = philox4x32_10(make_uint4(x1, t, kbase + (uint32_t)b1, 0u), tk.k0, tk.k1);
                const uint4 p2 = philox4x32_10(make_uint4(x2, t, kbase + (uint32_t)b2, 0u), tk.k0, tk.k1);
                ent[s1] = e1 | (p1.x & 0xC0000000u);
                uw[s1] = p1.y;
                if (two) {
                    ent[s2] = e2 | (p2.x & 0xC0000000u);
                    uw[s2] = p2.y;
                }
            }
            __syncthreads();
            if (tid < 4) s_count[tid] = 0;  // read by everyone above the barrier
            // B: the four classes in order
            int my_delta = 0;
#pragma unroll 1
            for (int b = 0; b < 4; ++b) {
                const int nbc = b == 0 ? n0 : b == 1 ? n1 : b == 2 ? n2 : n3;
                for (int e = tid; e < nbc; e += blockDim.x) {
                    const uint32_t en = ent[b * GQ + e];
                    const uint32_t u = uw[b * GQ + e];
                    const int m = (int)((en >> 16) & 0x3FFFu);
                    const int j = (int)(en & 0xFFFFu);
                    const int d = (int)(en >> 30);
                    uint32_t* rr = img + (rowbase + 4 * m - r0 + 3) * ldw;
                    const int c = j - 16;
                    const uint32_t wm3 = row_window(rr - 3 * ldw, L, c);
                    const uint32_t wm2 = row_window(rr - 2 * ldw, L, c);
                    const uint32_t wm1 = row_window(rr - ldw, L, c);
                    const uint32_t w00 = row_window(rr, L, c);
                    const uint32_t wp1 = row_window(rr + ldw, L, c);
                    const uint32_t wp2 = row_window(rr + 2 * ldw, L, c);
                    const uint32_t wp3 = row_window(rr + 3 * ldw, L, c);
                    const int o = dir_di(d);
                    const int p = 16 + dir_dj(d);
                    const uint32_t y2 = o < 0 ? wm3 : (o > 0 ? wm1 : wm2);
                    const uint32_t y1 = o < 0 ? wm2 : (o > 0 ? w00 : wm1);
                    const uint32_t y0 = o < 0 ? wm1 : (o > 0 ? wp1 : w00);
                    const uint32_t z1 = o < 0 ? w00 : (o > 0 ? wp2 : wp1);
                    const uint32_t z2 = o < 0 ? wp1 : (o > 0 ? wp3 : wp2);
                    const int sx = (int)((w00 >> 16) & 1u);
                    const int sy = (int)((y0 >> p) & 1u);
                    if (sx != sy) {
                        const int dsig = sigma_bits(wm2, wm1, w00, wp1, wp2, 16) -
                                         sigma_bits(y2, y1, y0, z1, z2, p);
                        if (u < sT[(dsig + 25) * 3 + (sx - sy + 1)]) {
                            atomicXor(&rr[j >> 5], 1u << (j & 31));
                            my_delta += sy ? 1 : -1;
                        }
                    }
                }
                __syncthreads();
            }
            if (my_delta) atomicAdd(&s_delta, my_delta);
            if (tk.drawn && tid == 0) atomicAdd(slot_of(tk.drawn, me), (unsigned long long)total);
        }

        // ---- publish the boundary rows of this step -----------------------
        if (!single) {
            uint64_t* slot = my_ring + (s & 1) * ringw;
            const uint64_t tag = (uint64_t)(uint32_t)(s + 1) << 32;
            for (int q = tid; q < 6 * nw; q += blockDim.x) {
                const int rr = q / nw, w = q - (q / nw) * nw;
                // ring rows 0..2: first 3 strip rows; 3..5: last 3 strip rows
                const uint32_t v = img[(rr < 3 ? 3 + rr : H - 3 + rr) * ldw + w];
                ring_store(slot + q, tag | v);
            }
        }
        __syncthreads();  // also orders the s_delta atomics before the read below
        if (tid == 0 && a == 3) {
            const int dsw = s_delta;
            s_delta = 0;
            if (dsw) atomicAdd(slot_of(tk.delta + (size_t)(s >> 2) * kSweepWords, me),
                               (unsigned long long)(long long)dsw);
        }
    }

    __syncthreads();
    for (int q = tid; q < H * nw; q += blockDim.x) {
        const int rr = q / nw, w = q - (q / nw) * nw;
        tk.lat[(size_t)(r0 + rr) * tk.stride + w] = img[(3 + rr) * ldw + w];
    }
}

__global__ void k_tasks_set(StripTask* tasks, int n_tasks, uint32_t t0, int n,
                            unsigned long long* delta, unsigned long long* drawn) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n_tasks) {
        tasks[q].t0 = t0;
        tasks[q].n = n;
        tasks[q].delta = delta;
        tasks[q].drawn = drawn;
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        p[q] = v;
}

hipError_t launch_tasks_set(StripTask* tasks, int n_tasks, uint32_t t0, int n,
                            unsigned long long* delta, unsigned long long* drawn, hipStream_t st) {
    hipLaunchKernelGGL(k_tasks_set, dim3((n_tasks + 255) / 256), dim3(256), 0, st, tasks, n_tasks, t0, n,
                       delta, drawn);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

size_t strip_lds_bytes(int L, int H, int G) {
    const int nw = (L + 31) / 32;
    const size_t words = 160 + (size_t)(H + 6) * (nw + 1) + 2 * (size_t)G * (nw + 1) +
                         8 * (size_t)G * (L / 4);
    return words * sizeof(uint32_t);
}

hipError_t launch_strip(const StripTask* d_tasks, int n_tasks, uint64_t* ring, uint32_t* abort_flag,
                        uint64_t wait_ticks, int G, size_t lds, hipStream_t st) {
    void* args[] = {(void*)&d_tasks, (void*)&n_tasks, (void*)&ring, (void*)&abort_flag,
                    (void*)&wait_ticks, (void*)&G};
    if (!allow_dynamic_lds((const void*)k_strip, lds)) return hipErrorInvalidValue;
    return hipLaunchCooperativeKernel((const void*)k_strip, dim3(n_tasks), dim3(kStripThreads), args,
                                      (unsigned int)lds, st);
}

hipError_t strip_capacity(size_t lds, int* blocks_per_cu, int* cus) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (!allow_dynamic_lds((const void*)k_strip, lds)) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void*)k_strip,
                                                        kStripThreads, lds);
}

}  // namespace pgg
