// Segment sweep on the bit-packed layout (gfx950): one wave per row segment,
// no workgroup barriers.  The kernel that launches it is k_ens_segment
// (pgg_ensemble.hip); a single lattice runs as a one-replica ensemble.
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
// discarded here.  A segment is at most L - 32 columns, or the whole row:
// then the margins hold the periodic images of owned sites, and an image is
// updated exactly as its original (same site index, so the same random
// numbers, and the same neighbourhood), so the owned columns stay exact.
//
// Per class the wave computes, bit-parallel over 32-bit words, the sites
// with a differing neighbour (the others cannot change and draw nothing),
// compacts them into a wave-private list, and processes the list: Philox
// block, payoff stencil, Fermi threshold, flip in LDS.  LDS operations of a
// wave complete in order, so the next class sees every flip of this one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pgg_device.hpp"
#include "pgg_internal.hpp"

namespace pgg {

namespace seg {

// 32 sites of a bit-packed row in global memory, columns c .. c + 31 taken
// modulo L (c any int >= -2L), column c in bit 0.  Reads only words < nw.
__device__ __forceinline__ uint32_t global_window(const uint32_t* __restrict__ row, int L, int nw, int c) {
    while (c < 0) c += L;
    while (c >= L) c -= L;
    if (c + 32 <= L) {
        const int w = c >> 5, sh = c & 31;
        const uint32_t lo = row[w];
        const uint32_t hi = sh ? row[w + 1] : 0u;  // c + 31 < L, so w + 1 < nw when sh > 0
        return funnel(hi, lo, sh);
    }
    uint32_t out = 0;
    int got = 0;
    while (got < 32) {
        const int take = min(32 - got, L - c);
        const int w = c >> 5, sh = c & 31;
        const uint32_t lo = row[w];
        const uint32_t hi = (sh && w + 1 < nw) ? row[w + 1] : 0u;
        uint32_t piece = funnel(hi, lo, sh);
        if (take < 32) piece &= (1u << take) - 1u;
        out |= piece << got;
        got += take;
        c = 0;
    }
    return out;
}

// The same 32 sites for L >= 32 and -L <= c < 2L, without loops: two loads
// and a funnel shift, and for a window that crosses column L - 1 the first
// columns of the row shifted in after it.
__device__ __forceinline__ uint32_t global_window_wide(const uint32_t* __restrict__ row, int L, int nw, int c) {
    c += (c < 0) ? L : 0;
    c -= (c >= L) ? L : 0;
    const int wi = c >> 5, sh = c & 31;
    const uint32_t lo = row[wi];
    const uint32_t hi = (wi + 1 < nw) ? row[wi + 1] : 0u;
    uint32_t v = funnel(hi, lo, sh);  // columns c, c + 1, ... of the stored words
    const int take = L - c;           // columns before the wrap (>= 1)
    if (take < 32) v = (v & ((1u << take) - 1u)) | (row[0] << take);
    return v;
}

// Sigma of the site in bit 16 of the middle row, without its 5 s term: the
// rows a2, a1, b, c1, c2 are i-2 .. i+2.  Sigma (the sum of the cooperator
// counts of the five groups containing the site) counts the site itself 5
// times, its 4 nearest neighbours twice, its 4 diagonal neighbours twice and
// the 4 sites at axis distance 2 once.
__device__ __forceinline__ int sigma_rest16(uint32_t a2, uint32_t a1, uint32_t b, uint32_t c1, uint32_t c2) {
    const int ones = __popc(b & 0x00044000u) + __popc(a2 & 0x00010000u) + __popc(c2 & 0x00010000u);
    const int twos = __popc(b & 0x00028000u) + __popc(a1 & 0x00038000u) + __popc(c1 & 0x00038000u);
    return ones + 2 * twos;
}

// Bits [lo, hi) of a 32-bit word (0 <= lo <= hi <= 32).
__device__ __forceinline__ uint32_t bit_range(int lo, int hi) {
    return (uint32_t)((1ull << hi) - (1ull << lo));
}

// Number of set bits of a wave-wide mask below the calling lane.
__device__ __forceinline__ int lanes_below(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

}  // namespace seg

// The threshold table in LDS, laid out for an index without a multiply:
// T[dSigma][ds] at word (ds + 1) * 64 + dSigma + 25 (three rows of 64 words,
// 51 used each).
constexpr int kSegTableWords = 192;

__device__ __forceinline__ void seg_load_table(uint32_t* __restrict__ sT, const uint32_t* __restrict__ T) {
    for (int k = threadIdx.x; k < kTableSize; k += blockDim.x) {
        const int dsig = k / 3, ds = k - 3 * dsig;  // T[(dSigma + 25) * 3 + ds + 1]
        sT[ds * 64 + dsig] = T[k];
    }
}

// Window words per row and list capacity per class for a segment width.
__host__ __device__ constexpr int seg_window_words(int segw) { return (segw + 31) / 32 + 4; }
// (class-b sites of a segment plus margins of up to 21 columns each side)
__host__ __device__ constexpr int seg_list_cap(int segw) { return segw / 4 + 16; }
__host__ __device__ constexpr int seg_wave_words(int segw) { return 7 * seg_window_words(segw) + seg_list_cap(segw); }

// The elementary step of the listed site at window position p of the row
// that rp points at (rows ld words apart, the window covering columns
// p - 16 .. p + 15 of the rows i - 3 .. i + 3), global site index x, sweep t,
// colour k: 0 if it keeps its strategy, else +1 (it becomes C) or -1 (D).
// Branch-free, so that two calls interleave.
__device__ __forceinline__ int site_step(const uint32_t* __restrict__ rp, int ld, int p, uint32_t x, uint32_t t,
                                         uint32_t k, uint32_t k0, uint32_t k1, const uint32_t* __restrict__ sT) {
    const uint2 rnd = philox4x32_10_w01(x, t, k, 0u, k0, k1);
    // neighbour y = x + (di, dj) for d = w0 >> 30: 0 E, 1 W, 2 S, 3 N
    const uint32_t d2 = (rnd.x >> 30) << 1;
    const int di = (int)__builtin_amdgcn_ubfe(0x25u, d2, 2u) - 1;
    const int dj = (int)__builtin_amdgcn_ubfe(0x52u, d2, 2u) - 1;
    // rows i-2 .. i+2 around x and around y, each a 32-column window with the
    // centre column in bit 16
    const int px = p - 16, py = px + dj;
    const uint32_t* rx = rp + (px >> 5);
    const uint32_t* ry = rp + __mul24(di, ld) + (py >> 5);
    const int shx = px & 31, shy = py & 31;
    const uint32_t xm2 = funnel(rx[1 - 2 * ld], rx[-2 * ld], shx);
    const uint32_t xm1 = funnel(rx[1 - ld], rx[-ld], shx);
    const uint32_t x0 = funnel(rx[1], rx[0], shx);
    const uint32_t xp1 = funnel(rx[1 + ld], rx[ld], shx);
    const uint32_t xp2 = funnel(rx[1 + 2 * ld], rx[2 * ld], shx);
    const uint32_t ym2 = funnel(ry[1 - 2 * ld], ry[-2 * ld], shy);
    const uint32_t ym1 = funnel(ry[1 - ld], ry[-ld], shy);
    const uint32_t y0 = funnel(ry[1], ry[0], shy);
    const uint32_t yp1 = funnel(ry[1 + ld], ry[ld], shy);
    const uint32_t yp2 = funnel(ry[1 + 2 * ld], ry[2 * ld], shy);
    const int sx = (int)((x0 >> 16) & 1u);
    const int sy = (int)((y0 >> 16) & 1u);
    const int ds = sx - sy;
    // Sigma = rest + 5 s, so Sigma_x - Sigma_y = rest_x - rest_y + 5 ds; the
    // index stays inside the table for ds = 0 too (rest lies in [0, 20])
    const int dsig = seg::sigma_rest16(xm2, xm1, x0, xp1, xp2) - seg::sigma_rest16(ym2, ym1, y0, yp1, yp2) + 5 * ds;
    const uint32_t thr = sT[((ds + 1) << 6) + dsig + 25];  // T[(dsig + 25) * 3 + ds + 1], seg_load_table's layout
    const bool flip = (ds != 0) & (rnd.y < thr);
    return flip ? (sy ? 1 : -1) : 0;
}

// Segment geometry of one wave: row i of residue a, owned columns [s, e),
// window bit 0 at column c0 = s - 64.
struct SegPos {
    int i, s, e, c0;
};

__device__ __forceinline__ SegPos seg_pos(int L, int a, int segw, int ri, int sg) {
    SegPos g;
    g.i = a + 4 * ri;
    g.s = sg * segw;
    g.e = min(L, g.s + segw);
    g.c0 = g.s - 64;
    return g;
}

// Fill the wave's LDS window with the 7 rows it reads (columns c0 .. c0 +
// 32 WB - 1, periodic).  The update is out of place: rows whose residue is
// below a are read from `next` (already updated in this sweep by an earlier
// launch), the others from `cur`; row i is later written to `next`.  So no
// wave reads a row that another wave of the same launch writes.  When L is
// a multiple of 32 every window word is one word of the row (segments start
// on word boundaries), and each lane issues its 7 loads back to back.
__device__ __forceinline__ void segment_fill(const uint32_t* __restrict__ cur, const uint32_t* __restrict__ next,
                                             int L, int stride, int nw, int a, int segw, const SegPos& g,
                                             uint32_t* __restrict__ win) {
    using namespace seg;
    const int lane = threadIdx.x & 63;
    const int WB = seg_window_words(segw);
    if ((L & 31) == 0) {
        const int w0 = (g.c0 >> 5);  // may be -2 or -1 for the first segment
        for (int wb = 0; wb < WB; wb += 64) {
            const int w = wb + lane;
            if (w < WB) {
                uint32_t v[7];
                int widx = w0 + w;                  // in [-2, nw + 2): one wrap suffices (nw >= 2)
                widx += (widx < 0) ? nw : 0;
                widx -= (widx >= nw) ? nw : 0;
#pragma unroll
                for (int o = 0; o < 7; ++o) {
                    int gi = g.i - 3 + o;
                    gi += (gi < 0) ? L : 0;
                    gi -= (gi >= L) ? L : 0;
                    const uint32_t* src = ((gi & 3) < a) ? next : cur;
                    v[o] = src[(size_t)gi * stride + widx];
                }
#pragma unroll
                for (int o = 0; o < 7; ++o) win[o * WB + w] = v[o];
            }
        }
        return;
    }
    // L not a multiple of 32: each window word is columns c .. c + 31 of
    // its row, modulo L (c0 >= -64 and the window ends before column 2L)
    for (int wb = 0; wb < WB; wb += 64) {
        const int w = wb + lane;
        if (w < WB) {
            const int c = g.c0 + 32 * w;
            uint32_t v[7];
#pragma unroll
            for (int o = 0; o < 7; ++o) {
                int gi = g.i - 3 + o;
                gi += (gi < 0) ? L : 0;
                gi -= (gi >= L) ? L : 0;
                const uint32_t* src = ((gi & 3) < a) ? next : cur;
                v[o] = global_window_wide(src + (size_t)gi * stride, L, nw, c);
            }
#pragma unroll
            for (int o = 0; o < 7; ++o) win[o * WB + w] = v[o];
        }
    }
}

// The four colour classes on the filled window, then the owned columns
// written to next.  sT: the threshold table in LDS.  Adds the net change of
// the cooperator count over the owned columns to my_delta (every lane) and
// the number of draws of owned sites to my_drawn (per lane; the caller sums
// over the wave).
//
// r0: the row's window (rows r0 - 3 WB .. r0 + 3 WB hold rows i-3 .. i+3);
// list: seg_list_cap(segw) words of the wave's own.  extra widens every
// class's margin (a launch that runs a second residue after this one needs
// this row exact on 3 x 4 more columns each side).  A row that is not owned
// (a halo row another workgroup owns) is updated in LDS only: no counts, no
// write-back.  Draws are counted only when count_drawn is set (wave-uniform;
// the count is a diagnostic).
__device__ __forceinline__ void segment_run_row(uint32_t* __restrict__ next, int L, int stride, int a, int segw,
                                                const SegPos& g, uint32_t t, uint32_t k0, uint32_t k1,
                                                const uint32_t* __restrict__ sT, uint32_t* __restrict__ r0,
                                                uint32_t* __restrict__ list, int extra, bool owned_row,
                                                bool count_drawn, int& my_delta, int& my_drawn) {
    using namespace seg;
    const int lane = threadIdx.x & 63;
    const int WB = seg_window_words(segw);
    const int i = g.i, s = g.s, e = g.e, c0 = g.c0;
    __builtin_amdgcn_wave_barrier();

    const uint32_t k_first = (uint32_t)(4 * a);
#pragma unroll 1
    for (int b = 0; b < 4; ++b) {
        // Class-b sites on window positions [lo, hi).
        const int m = extra + 9 - 3 * b;
        const int lo = 64 - m, hi = 64 + (e - s) + m;
        const int wlo = lo >> 5, whi = (hi + 31) >> 5;
        // 1. candidates per word (the class-b bits), 2. compacted list: each
        // lane's offset is the exclusive prefix sum of the candidate counts
        // of the lanes below it, taken bit-sliced from ballots.
        // positions [lo, hi): only the first and the last word are partial
        const uint32_t m_first = 0xFFFFFFFFu << (lo & 31);
        const uint32_t m_last = (hi & 31) ? (1u << (hi & 31)) - 1u : 0xFFFFFFFFu;
        auto word_act = [&](int w) {
            const uint32_t X = r0[w];
            const uint32_t E = funnel(r0[w + 1], X, 1);
            const uint32_t Wn = funnel(X, r0[w - 1], 31);
            uint32_t act = ((X ^ E) | (X ^ Wn) | (X ^ r0[w - WB]) | (X ^ r0[w + WB])) & (0x11111111u << b);
            if (w == wlo) act &= m_first;
            if (w == whi - 1) act &= m_last;
            // draws of owned sites (margin sites are recomputed copies)
            if (count_drawn && owned_row) {
                const int own_lo = max(64 - 32 * w, 0), own_hi = min(64 + (e - s) - 32 * w, 32);
                if (own_hi > own_lo) my_drawn += __popc(act & bit_range(own_lo, own_hi));
            }
            return act;
        };
        // Up to 128 words per pass, lane l taking words wbase + l and wbase +
        // 64 + l: a row a little over 64 words (2048 owned columns and their
        // margins) takes one pass, its last few words loaded and listed
        // beside the first 64 instead of in a pass of their own.
        int total = 0;  // wave-uniform
        // this lane's offset: the counts (0..2^nbits - 1) of the lanes below
        auto offset = [&](int cnt, int nbits) {
            int pos = total;
            for (int k = 0; k < nbits; ++k) {
                const unsigned long long m = __ballot((cnt >> k) & 1);
                pos += lanes_below(m) << k;
                total += __popcll(m) << k;
            }
            return pos;
        };
        auto emit = [&](uint32_t act, int w, int& pos) {
            while (act) {
                const int bit = __ffs(act) - 1;
                act &= act - 1u;
                list[pos++] = (uint32_t)(32 * w + bit);
            }
        };
        for (int wbase = wlo; wbase < whi; wbase += 128) {
            const int w1 = wbase + lane, w2 = w1 + 64;
            if (wbase + 64 < whi) {  // wave-uniform: two words for some lanes
                const uint32_t act1 = word_act(w1);  // w1 < wbase + 64 < whi
                const uint32_t act2 = w2 < whi ? word_act(w2) : 0u;
                int pos = offset(__popc(act1) + __popc(act2), 5);
                emit(act1, w1, pos);
                emit(act2, w2, pos);
            } else {
                const uint32_t act1 = w1 < whi ? word_act(w1) : 0u;
                int pos = offset(__popc(act1), 4);
                emit(act1, w1, pos);
            }
        }
        __builtin_amdgcn_wave_barrier();
        // 3. the elementary steps of the listed sites, two per lane per step
        // (both decided before either flips: sites of one class never read
        // each other's strategy).
        const uint32_t k = k_first + (uint32_t)b;
        const uint32_t row_base = (uint32_t)(i * L);
        auto site_of = [&](int p) {
            // column c0 + p modulo L (it lies in [-L, 2L)): the least of c,
            // c + L and c - L taken as unsigned numbers
            const uint32_t c = (uint32_t)(c0 + p);
            return row_base + min(min(c, c + (uint32_t)L), c - (uint32_t)L);
        };
        auto apply = [&](int p, int f) {
            atomicXor(&r0[p >> 5], 1u << (p & 31));
            if (owned_row && p >= 64 && p < 64 + (e - s)) my_delta += f;
        };
        for (int qb = 0; qb < total; qb += 128) {
            const int q1 = qb + lane, q2 = q1 + 64;
            if (qb + 64 < total) {  // wave-uniform: some lanes have a second entry
                const int p1 = (int)list[min(q1, total - 1)];
                const int p2 = (int)list[min(q2, total - 1)];
                const int f1 = site_step(r0, WB, p1, site_of(p1), t, k, k0, k1, sT);
                const int f2 = site_step(r0, WB, p2, site_of(p2), t, k, k0, k1, sT);
                if (q1 < total && f1) apply(p1, f1);
                if (q2 < total && f2) apply(p2, f2);
            } else if (q1 < total) {
                const int p1 = (int)list[q1];
                const int f1 = site_step(r0, WB, p1, site_of(p1), t, k, k0, k1, sT);
                if (f1) apply(p1, f1);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }

    // Write back the owned columns [s, e): window words 2 .. 2 + ceil((e-s)/32).
    if (!owned_row) return;
    const int nown = (e - s + 31) >> 5;
    for (int q = lane; q < nown; q += 64) {
        uint32_t v = r0[2 + q];
        const int valid = e - (s + 32 * q);
        if (valid < 32) v &= (1u << valid) - 1u;
        next[(size_t)i * stride + (s >> 5) + q] = v;
    }
}

// One wave's segment with its private 7-row window (win: 7 WB words, then
// the list).
__device__ __forceinline__ void segment_run(uint32_t* __restrict__ next, int L, int stride, int a, int segw,
                                            const SegPos& g, uint32_t t, uint32_t k0, uint32_t k1,
                                            const uint32_t* __restrict__ sT, uint32_t* __restrict__ win,
                                            bool count_drawn, int& my_delta, int& my_drawn) {
    const int WB = seg_window_words(segw);
    segment_run_row(next, L, stride, a, segw, g, t, k0, k1, sT, win + 3 * WB, win + 7 * WB, 0, true, count_drawn,
                    my_delta, my_drawn);
}

}  // namespace pgg
