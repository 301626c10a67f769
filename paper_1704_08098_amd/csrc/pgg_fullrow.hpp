// Full-row sweep on the bit-packed layout (gfx950): one wave owns R whole
// rows of the launch's residue a (rows i0, i0 + 4, ..., i0 + 4 (R - 1)),
// for L a multiple of 32.  Owning whole rows, the wave needs no column
// margins and recomputes nothing: the classes 4a..4a+3 run on the full
// periodic rows.  Small lattices take several rows per wave so that a
// class still lists enough sites to fill a 64-lane pass.
//
// The wave's LDS window holds rows i0 - 3 .. i0 + 4 (R - 1) + 3 (4R + 3 rows,
// periodic), each as its nw = L / 32 words plus one pad word on each side
// that repeats the word across the wrap (pad left = word nw - 1, pad right =
// word 0), so neighbour and stencil windows never index modulo L.  Only the
// owned rows change in a launch, and a flip in word 0 or nw - 1 is applied
// to the pad copy as well.  A row of residue a never reads another row of
// residue a (they are 4 apart, the stencil reaches 3), so copies of a row
// that the window holds twice (R = L / 4) are never read stale.
// Same update rule, lists and out-of-place double buffering as the segment
// sweep (pgg_segment.hpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pgg_device.hpp"
#include "pgg_internal.hpp"
#include "pgg_segment.hpp"

namespace pgg {

// Words of a full-row wave's LDS: the window rows, then one class list.
__host__ __device__ constexpr int fr_window_ldw(int L) { return L / 32 + 2; }
__host__ __device__ constexpr int fr_wave_words(int L, int R) {
    return (4 * R + 3) * fr_window_ldw(L) + R * (L / 4) + 8;
}

// LDS words one wave of this replica uses (whole rows or a segment).
__host__ __device__ inline int rep_wave_words(const EnsRep& rp) {
    return rp.rpw > 0 ? fr_wave_words(rp.L, rp.rpw) : seg_wave_words(rp.segw);
}

// Fill the window: rows of residue below a from next (updated earlier in
// this sweep), the others from cur.
__device__ __forceinline__ void fullrow_fill(const uint32_t* __restrict__ cur, const uint32_t* __restrict__ next,
                                             int L, int stride, int a, int i0, int R, uint32_t* __restrict__ win) {
    const int lane = threadIdx.x & 63;
    const int nw = L >> 5, ldw = nw + 2;
    const int n = (4 * R + 3) * ldw;
    // four loads in flight per lane before their LDS stores: one round trip
    // to L2 per 256 words of the window, not one per 64
    constexpr int U = 4;
    for (int qb = 0; qb < n; qb += 64 * U) {
        uint32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = qb + 64 * u + lane;
            v[u] = 0u;
            if (q < n) {
                const int o = q / ldw;
                int w = q - o * ldw - 1;  // -1 .. nw
                w += (w < 0) ? nw : 0;
                w -= (w >= nw) ? nw : 0;
                int gi = i0 - 3 + o;  // in [-3, 2L)
                gi += (gi < 0) ? L : 0;
                gi -= (gi >= L) ? L : 0;
                const uint32_t* src = ((gi & 3) < a) ? next : cur;
                v[u] = src[(size_t)gi * stride + w];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = qb + 64 * u + lane;
            if (q < n) win[q] = v[u];
        }
    }
}

// The four classes on the nrows (<= R) owned rows, then the rows written to
// next (next == nullptr: no write-back, the rows stay in LDS).  Adds the net
// change of the cooperator count to my_delta (every lane) and the number of
// draws to my_drawn (per lane; the caller sums over the wave).  list: the
// class list (R L / 4 + 8 words), or nullptr for the words after the window.
__device__ __forceinline__ void fullrow_run(uint32_t* __restrict__ next, int L, int stride, int a, int i0, int R,
                                            int nrows, uint32_t t, uint32_t k0, uint32_t k1,
                                            const uint32_t* __restrict__ sT, uint32_t* __restrict__ win,
                                            int& my_delta, int& my_drawn, uint32_t* __restrict__ list_in = nullptr) {
    const int lane = threadIdx.x & 63;
    const int nw = L >> 5, ldw = nw + 2;
    uint32_t* list = list_in ? list_in : win + (4 * R + 3) * ldw;
    uint32_t* row0 = win + 3 * ldw + 1;  // word 0 of owned row 0; owned row r starts 4 ldw later per r
    const int nwords = nrows * nw;
    const uint32_t k_first = (uint32_t)(4 * a);
    __builtin_amdgcn_wave_barrier();
#pragma unroll 1
    for (int b = 0; b < 4; ++b) {
        // 1. candidates: class-b sites with a differing neighbour, per word
        int total = 0;  // wave-uniform
        for (int qb = 0; qb < nwords; qb += 64) {
            const int q = qb + lane;
            uint32_t act = 0;
            int r = 0, w = 0;
            if (q < nwords) {
                r = q / nw;
                w = q - r * nw;
                const uint32_t* rp = row0 + 4 * r * ldw;
                const uint32_t X = rp[w];
                const uint32_t E = funnel(rp[w + 1], X, 1);
                const uint32_t Wn = funnel(X, rp[w - 1], 31);
                act = ((X ^ E) | (X ^ Wn) | (X ^ rp[w - ldw]) | (X ^ rp[w + ldw])) & (0x11111111u << b);
            }
            // 2. compacted list: entry = r << 16 | column
            const int cnt = __popc(act);
            my_drawn += cnt;
            int pos = total;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const unsigned long long m = __ballot((cnt >> k) & 1);
                pos += seg::lanes_below(m) << k;
                total += __popcll(m) << k;
            }
            const uint32_t tag = ((uint32_t)r << 16) | (uint32_t)(32 * w);
            while (act) {
                const int bit = __ffs(act) - 1;
                act &= act - 1u;
                list[pos++] = tag | (uint32_t)bit;
            }
        }
        __builtin_amdgcn_wave_barrier();
        // 3. the elementary steps of the listed sites, two per lane per step
        // (both decided before either flips: sites of one class never read
        // each other's strategy).  Columns p - 16 .. p + 15 lie within the
        // pad words.
        const uint32_t k = k_first + (uint32_t)b;
        auto step = [&](uint32_t en) {
            const int r = (int)(en >> 16), p = (int)(en & 0xFFFFu);
            return site_step(row0 + 4 * r * ldw, ldw, p, (uint32_t)((i0 + 4 * r) * L + p), t, k, k0, k1, sT);
        };
        auto apply = [&](uint32_t en, int f) {
            const int r = (int)(en >> 16), p = (int)(en & 0xFFFFu);
            uint32_t* rp = row0 + 4 * r * ldw;
            const int wx = p >> 5;
            const uint32_t bit = 1u << (p & 31);
            atomicXor(&rp[wx], bit);
            if (wx == 0) atomicXor(&rp[nw], bit);       // right pad repeats word 0
            if (wx == nw - 1) atomicXor(&rp[-1], bit);  // left pad repeats word nw - 1
            my_delta += f;
        };
        for (int qb = 0; qb < total; qb += 128) {
            const int q1 = qb + lane, q2 = q1 + 64;
            if (qb + 64 < total) {  // wave-uniform: some lanes have a second entry
                const uint32_t e1 = list[min(q1, total - 1)], e2 = list[min(q2, total - 1)];
                const int f1 = step(e1), f2 = step(e2);
                if (q1 < total && f1) apply(e1, f1);
                if (q2 < total && f2) apply(e2, f2);
            } else if (q1 < total) {
                const uint32_t e1 = list[q1];
                const int f1 = step(e1);
                if (f1) apply(e1, f1);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    // Write back the owned rows.
    if (!next) return;
    for (int q = lane; q < nwords; q += 64) {
        const int r = q / nw, w = q - r * nw;
        next[(size_t)(i0 + 4 * r) * stride + w] = row0[4 * r * ldw + w];
    }
}

}  // namespace pgg
