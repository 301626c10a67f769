// Segment sweep on the bit-packed layout (gfx950): one wave per row segment,
// no workgroup barriers.
//
// One launch per row residue a = i mod 4 runs the colour classes
// k = 4a + 0..3.  Within such a launch only the rows with i mod 4 = a change,
// each only through its own sites, and a site reads rows i-3..i+3 and
// columns j-3..j+3.  So a row can be cut into segments [s, e) that are
// processed independently: the wave owning a segment copies the 7 rows it
// reads into a private LDS window (columns s-64 .. e+63, periodic), and
// updates class b on the columns [s - m_b, e + m_b) with m = (9, 6, 3, 0):
// class 3 on [s, e) reads classes 0-2 only within 3 columns, class 2 on
// [s-3, e+3) reads classes 0-1 within 3 more, and so on, so every site the
// wave writes back -- the columns [s, e) -- is exact.  Sites in the margins
// are recomputed (identically) by the neighbouring segment's wave and
// discarded here.  A segment is at most half a row, so a margin site and
// its periodic image never both lie in the columns read.
//
// Per class the wave computes, bit-parallel over 32-bit words, the sites
// with a differing neighbour (the others cannot change and draw nothing),
// compacts them into a wave-private list, and processes the list: Philox
// block, payoff stencil, Fermi threshold, flip in LDS.  LDS operations of a
// wave complete in order, so the next class sees every flip of this one.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pgg_segment.hpp"

namespace pgg {

__global__ void __launch_bounds__(kSegmentThreads)
k_segment(const uint32_t* __restrict__ cur, uint32_t* __restrict__ next, int L, int stride, int nw, int a,
          int segw, int nseg, uint32_t t,
          uint32_t k0, uint32_t k1, const uint32_t* __restrict__ T, unsigned long long* __restrict__ delta,
          unsigned long long* __restrict__ drawn) {
    extern __shared__ uint32_t smem[];
    __shared__ int s_part[2 * (kSegmentThreads / 64)];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    uint32_t* sT = smem;
    uint32_t* win = smem + 160 + wid * seg_wave_words(segw);

    for (int q = threadIdx.x; q < kTableSize; q += blockDim.x) sT[q] = T[q];
    __syncthreads();  // the table is shared by the workgroup's waves

    const int gw = blockIdx.x * (kSegmentThreads / 64) + wid;  // global wave index
    int my_delta = 0, my_drawn = 0;
    if (gw < (L >> 2) * nseg) {  // waves past the last segment only join the reduction
        const int ri = gw / nseg, sg = gw - (gw / nseg) * nseg;
        segment_wave(cur, next, L, stride, nw, a, segw, ri, sg, t, k0, k1, sT, win, my_delta, my_drawn);
    }
    // Reduce over the workgroup; one atomic per workgroup on a spread slot.
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) my_delta += __shfl_xor(my_delta, off, 64);
    if (lane == 0) {
        s_part[wid] = my_delta;
        s_part[kSegmentThreads / 64 + wid] = my_drawn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int dsum = 0, nsum = 0;
        for (int q = 0; q < kSegmentThreads / 64; ++q) {
            dsum += s_part[q];
            nsum += s_part[kSegmentThreads / 64 + q];
        }
        if (dsum) atomicAdd(slot_of(delta, (int)blockIdx.x), (unsigned long long)(long long)dsum);
        if (drawn && nsum) atomicAdd(slot_of(drawn, (int)blockIdx.x), (unsigned long long)nsum);
    }
}

size_t segment_lds_bytes(int segw) {
    return (160 + (size_t)(kSegmentThreads / 64) * seg_wave_words(segw)) * sizeof(uint32_t);
}

hipError_t launch_segment_residue(const uint32_t* cur, uint32_t* next, int L, int stride, int segw, int a, uint32_t t,
                                  uint64_t seed, const uint32_t* T, unsigned long long* delta,
                                  unsigned long long* drawn, hipStream_t st) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int nw = (L + 31) / 32;
    const int nseg = (L + segw - 1) / segw;
    const int waves = (L / 4) * nseg;
    const int wpb = kSegmentThreads / 64;
    const int blocks = (waves + wpb - 1) / wpb;
    hipLaunchKernelGGL(k_segment, dim3(blocks), dim3(kSegmentThreads), segment_lds_bytes(segw), st, cur, next,
                       L, stride, nw, a, segw, nseg, t, k0, k1, T, delta, drawn);
    return hipGetLastError();
}

}  // namespace pgg
