// Staged row-band sweep on the bit-packed layout (gfx950).
//
// Same work split as the row-band kernel (one launch per row residue a runs
// the colour classes k = 4a + 0..3 on rows staged in LDS), but the random
// numbers of all four classes are drawn in one barrier-free batch before the
// first class is updated, so the Philox work of a launch is spread over all
// lanes instead of being serialised by the three barriers between classes.
//
// Which sites draw: a site's elementary step can only change it if one of
// its four neighbours holds the other strategy (copying an equal strategy is
// a no-op, and the counter-based generator needs no draw to stay in step).
// At the time of class b, a site and its N/S neighbours (rows of another
// residue) still hold their launch-start values; of its E/W neighbours only
// the one updated earlier in this launch can have changed -- the W neighbour
// (class b-1) for b >= 1, and for b = 3 also the E neighbour (class 0) --
// and only if that neighbour could itself change.  So
//     C0 = A & class0,  C1 = (A | C0 << 1) & class1,  C2 = (A | C1 << 1) & class2,
//     C3 = (A | C2 << 1 | C0 >> 1) & class3,
// with A the sites that differ from a neighbour at launch start and shifts
// along the periodic row, contains every site that can change.  Only the
// sites of C0..C3 draw; the update itself re-reads the current strategies,
// so the result is the same as drawing for every site.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pgg_device.hpp"
#include "pgg_internal.hpp"

namespace pgg {

__global__ void __launch_bounds__(kRowbandThreads)
k_rowband_staged(uint32_t* __restrict__ lat, int L, int stride, int nw, int a, int R, uint32_t t,
                 uint32_t k0, uint32_t k1, const uint32_t* __restrict__ T,
                 unsigned long long* __restrict__ delta, unsigned long long* __restrict__ drawn) {
    extern __shared__ uint32_t smem[];
    const int ldw = nw + 1;  // one zero pad word per staged row
    const int q4 = L >> 2;   // sites per row per colour class
    const int RQ = R * q4;   // list capacity per class
    uint32_t* sT = smem;                       // kTableSize (padded to 160)
    uint32_t* img = sT + 160;                  // (4R + 3) rows
    uint32_t* c0row = img + (4 * R + 3) * ldw; // R rows: class-0 candidates
    uint32_t* actrow = c0row + R * ldw;        // R rows: launch-start activity
    uint32_t* ent = actrow + R * ldw;          // 4 * RQ entries: (d << 30) | (m << 16) | j
    uint32_t* uw = ent + 4 * RQ;               // 4 * RQ acceptance words
    __shared__ int s_count[4];
    __shared__ int s_delta;

    const int g = blockIdx.x;
    const int i0 = a + 4 * R * g;
    const int Rv = min(R, q4 - g * R);
    const int tid = threadIdx.x;

    for (int q = tid; q < kTableSize; q += blockDim.x) sT[q] = T[q];
    if (tid < 4) s_count[tid] = 0;
    if (tid == 0) s_delta = 0;
    const int nrows = 4 * Rv + 3;
    for (int q = tid; q < nrows * ldw; q += blockDim.x) {
        const int rho = q / ldw, w = q - (q / ldw) * ldw;
        int gi = i0 - 3 + rho;
        gi += (gi < 0) ? L : 0;
        gi -= (gi >= L) ? L : 0;
        img[q] = (w < nw) ? lat[(size_t)gi * stride + w] : 0u;
    }
    __syncthreads();

    // Stage A1: launch-start activity and class-0 candidates, per word.
    for (int q = tid; q < Rv * ldw; q += blockDim.x) {
        const int m = q / ldw, w = q - (q / ldw) * ldw;
        uint32_t act = 0;
        if (w < nw) {
            const uint32_t* r0 = img + (3 + 4 * m) * ldw;
            const uint32_t X = r0[w];
            const uint32_t E = row_window(r0, L, 32 * w + 1);
            const uint32_t Wn = row_window(r0, L, 32 * w - 1);
            const int valid = L - 32 * w;
            const uint32_t vmask = valid >= 32 ? 0xFFFFFFFFu : ((1u << valid) - 1u);
            act = ((X ^ E) | (X ^ Wn) | (X ^ r0[w - ldw]) | (X ^ r0[w + ldw])) & vmask;
        }
        actrow[q] = act;
        c0row[q] = act & 0x11111111u;
    }
    __syncthreads();

    // Stage A2: classes 1..3 and the per-class candidate lists.
    for (int q = tid; q < Rv * nw; q += blockDim.x) {
        const int m = q / nw, w = q - (q / nw) * nw;
        const uint32_t act = actrow[m * ldw + w];
        const uint32_t c0 = c0row[m * ldw + w];
        const uint32_t c1 = (act | (c0 << 1)) & 0x22222222u;
        const uint32_t c2 = (act | (c1 << 1)) & 0x44444444u;
        // C0 at column j + 1; the window wraps past column L - 1, so keep
        // only the columns of the row.
        const int valid = L - 32 * w;
        const uint32_t vmask = valid >= 32 ? 0xFFFFFFFFu : ((1u << valid) - 1u);
        const uint32_t e0 = row_window(c0row + m * ldw, L, 32 * w + 1) & vmask;
        const uint32_t c3 = (act | (c2 << 1) | e0) & 0x88888888u;
        const uint32_t cls[4] = {c0, c1, c2, c3};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            uint32_t bits = cls[b];
            const int cnt = __popc(bits);
            if (cnt) {
                int pos = atomicAdd(&s_count[b], cnt);
                uint32_t* dst = ent + b * RQ;
                while (bits) {
                    const int bit = __ffs(bits) - 1;
                    bits &= bits - 1u;
                    dst[pos++] = ((uint32_t)m << 16) | (uint32_t)(32 * w + bit);
                }
            }
        }
    }
    __syncthreads();

    // Stage A3: the random numbers of every candidate of the four classes,
    // two independent Philox blocks per lane per iteration.
    const int n0 = s_count[0], n1 = s_count[1], n2 = s_count[2], n3 = s_count[3];
    const int total = n0 + n1 + n2 + n3;
    const uint32_t kbase = (uint32_t)(4 * a);
    auto list_slot = [&](int f, int& b) {
        b = (f >= n0) + (f >= n0 + n1) + (f >= n0 + n1 + n2);
        const int off = b == 0 ? 0 : b == 1 ? n0 : b == 2 ? n0 + n1 : n0 + n1 + n2;
        return b * RQ + (f - off);
    };
    for (int f = tid; f < total; f += 2 * (int)blockDim.x) {
        const int f2 = f + (int)blockDim.x;
        const bool two = f2 < total;
        int b1, b2;
        const int s1 = list_slot(f, b1);
        const int s2 = list_slot(two ? f2 : f, b2);
        const uint32_t e1 = ent[s1], e2 = ent[s2];
        const uint32_t x1 = (uint32_t)(i0 + 4 * (int)(e1 >> 16)) * (uint32_t)L + (e1 & 0xFFFFu);
        const uint32_t x2 = (uint32_t)(i0 + 4 * (int)(e2 >> 16)) * (uint32_t)L + (e2 & 0xFFFFu);
        const uint4 r1 = philox4x32_10(make_uint4(x1, t, kbase + (uint32_t)b1, 0u), k0, k1);
        const uint4 r2 = philox4x32_10(make_uint4(x2, t, kbase + (uint32_t)b2, 0u), k0, k1);
        ent[s1] = e1 | (r1.x & 0xC0000000u);
        uw[s1] = r1.y;
        if (two) {
            ent[s2] = e2 | (r2.x & 0xC0000000u);
            uw[s2] = r2.y;
        }
    }
    __syncthreads();

    // Stage B: the four classes in order; only the payoff stencil remains.
    int my_delta = 0;
#pragma unroll 1
    for (int b = 0; b < 4; ++b) {
        const int nbc = b == 0 ? n0 : b == 1 ? n1 : b == 2 ? n2 : n3;
        for (int e = tid; e < nbc; e += blockDim.x) {
            const uint32_t en = ent[b * RQ + e];
            const uint32_t u = uw[b * RQ + e];
            const int m = (int)((en >> 16) & 0x3FFFu);
            const int j = (int)(en & 0xFFFFu);
            const int d = (int)(en >> 30);
            uint32_t* r0 = img + (3 + 4 * m) * ldw;
            const int c = j - 16;
            const uint32_t wm3 = row_window(r0 - 3 * ldw, L, c);
            const uint32_t wm2 = row_window(r0 - 2 * ldw, L, c);
            const uint32_t wm1 = row_window(r0 - ldw, L, c);
            const uint32_t w00 = row_window(r0, L, c);
            const uint32_t wp1 = row_window(r0 + ldw, L, c);
            const uint32_t wp2 = row_window(r0 + 2 * ldw, L, c);
            const uint32_t wp3 = row_window(r0 + 3 * ldw, L, c);
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
                const int dsig = sigma_bits(wm2, wm1, w00, wp1, wp2, 16) - sigma_bits(y2, y1, y0, z1, z2, p);
                if (u < sT[(dsig + 25) * 3 + (sx - sy + 1)]) {
                    atomicXor(&r0[j >> 5], 1u << (j & 31));
                    my_delta += sy ? 1 : -1;
                }
            }
        }
        __syncthreads();
    }

    for (int q = tid; q < Rv * nw; q += blockDim.x) {
        const int m = q / nw, w = q - (q / nw) * nw;
        lat[(size_t)(i0 + 4 * m) * stride + w] = img[(3 + 4 * m) * ldw + w];
    }
    if (my_delta) atomicAdd(&s_delta, my_delta);
    __syncthreads();
    if (tid == 0) {
        if (s_delta) atomicAdd(slot_of(delta, (int)blockIdx.x), (unsigned long long)(long long)s_delta);
        if (drawn) atomicAdd(slot_of(drawn, (int)blockIdx.x), (unsigned long long)total);
    }
}

size_t staged_lds_bytes(int L, int R) {
    const int nw = (L + 31) / 32;
    const size_t words = 160 + (size_t)(4 * R + 3) * (nw + 1) + 2 * (size_t)R * (nw + 1) +
                         8 * (size_t)R * (L / 4);
    return words * sizeof(uint32_t);
}

hipError_t launch_staged_residue(uint32_t* lat, int L, int stride, int R, int a, uint32_t t,
                                 uint64_t seed, const uint32_t* T, unsigned long long* delta,
                                 unsigned long long* drawn, hipStream_t st) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int nw = (L + 31) / 32;
    const int bands = (L / 4 + R - 1) / R;
    if (!allow_dynamic_lds((const void*)k_rowband_staged, staged_lds_bytes(L, R))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rowband_staged, dim3(bands), dim3(kRowbandThreads), staged_lds_bytes(L, R), st,
                       lat, L, stride, nw, a, R, t, k0, k1, T, delta, drawn);
    return hipGetLastError();
}

}  // namespace pgg
