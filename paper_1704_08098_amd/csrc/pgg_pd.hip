// The pairwise prisoner's dilemma that Sec. VI names as the next game for the
// same scheme: each player plays the four nearest neighbours pairwise (weak
// dilemma: R = 1 for C meeting C, T = b for D meeting C, S = P = 0) and
// imitates a random neighbour with the Fermi probability of Eq. (3).  A
// player with n cooperating neighbours earns n as a cooperator and b n as a
// defector, so the acceptance threshold is a function of (s_x, n_x, n_y): 50
// entries built once on the host.
//
// An elementary step of x reads the radius-2 diamond around it (one line
// less than the public goods game).  The sweep runs 8 colour classes, the
// cosets of the sublattice spanned by (2, 2) and (4, 0): class k = 4 (i mod 2)
// + ((j - 2 h) mod 4), h = (i div 2) mod 2, in ascending order.  Same-class
// sites are at least 4 apart, so a class updates in parallel.
//
// One launch per class: a thread owns one 32-column word of one row of the
// class's row parity.  It reads 64-bit windows (columns 32 w - 16 .. 32 w +
// 47) of the five rows i-2 .. i+2 and finds the class sites of its word with
// a differing neighbour (the others cannot change and draw nothing).  The
// wave's sites are compacted into one list in LDS, beside every lane's
// windows, and the lanes then take the list one site each per pass: Philox
// block of counter (x, t, k, 0), the rule, the flip into the owner's word in
// LDS.  Every bit read outside the word's class sites is a site of another
// class, unchanged during the launch, so the order in which sites are
// decided never matters; each thread writes only its own word.
#include <hip/hip_runtime.h>

#include <cmath>
#include <stdint.h>

#include "pgg_device.hpp"
#include "pgg_internal.hpp"
#include "pgg_segment.hpp"

namespace pgg {

constexpr int kPdThreads = 256;

// The thresholds of the pairwise game for temptation b and noise K:
// T[(dir * 5 + n_x) * 5 + n_y], dir 0 = x cooperates and copies a defector
// (Pi_x = n_x, Pi_y = b n_y), dir 1 = x defects and copies a cooperator
// (Pi_x = b n_x, Pi_y = n_y); W = 1 / (1 + exp((Pi_x - Pi_y) / K)) and
// T = min(2^32 - 1, floor(W 2^32 + 1/2)).  binary64, host libm exp, fixed
// operation order.
void pd_table(double b, double K, uint32_t* T) {
#pragma clang fp contract(off)
    for (int idx = 0; idx < kPdTableSize; ++idx) {
        const int dir = idx / 25, nx = (idx / 5) % 5, ny = idx % 5;
        const double pix = dir == 0 ? 1.0 * (double)nx : b * (double)nx;
        const double piy = dir == 0 ? b * (double)ny : 1.0 * (double)ny;
        const double w = 1.0 / (1.0 + std::exp((pix - piy) / K));
        const double scaled = std::floor(w * 4294967296.0 + 0.5);
        T[idx] = scaled >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)scaled;
    }
}

__device__ __forceinline__ uint32_t bit64(uint64_t v, int p) { return (uint32_t)(v >> p) & 1u; }

// Per wave in LDS: every lane's five windows and its row base, the lanes'
// words (flips land there), and the class list of the wave.
constexpr int kPdWaves = kPdThreads / 64;
constexpr int kPdLaneWords = 11;                    // 5 x (lo, hi) windows, row base
constexpr int kPdWaveWords = 64 * kPdLaneWords + 64 + 64 * 8;

__global__ void __launch_bounds__(kPdThreads)
k_pd_class(uint32_t* __restrict__ lat, int L, int stride, int nw, int k, uint32_t t, uint32_t k0, uint32_t k1,
           const uint32_t* __restrict__ T, unsigned long long* __restrict__ delta) {
    __shared__ uint32_t sT[kPdTableSize];
    __shared__ int s_part[kPdWaves];
    __shared__ uint32_t s_wave[kPdWaves * kPdWaveWords];
    for (int q = threadIdx.x; q < kPdTableSize; q += blockDim.x) sT[q] = T[q];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t* lw = s_wave + wid * kPdWaveWords;  // lane windows: lane * kPdLaneWords
    uint32_t* words = lw + 64 * kPdLaneWords;     // the lanes' words
    uint32_t* list = words + 64;                  // entries lane << 5 | bit
    const int p = k >> 2, qc = k & 3;
    const int rows = L >> 1;  // rows of parity p
    const int64_t task = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t act = 0, own = 0;
    int ri = 0, w = 0;
    if (task < (int64_t)rows * nw) {
        ri = (int)(task / nw);
        w = (int)(task - (int64_t)ri * nw);
        const int i = p + 2 * ri;
        const int h = (i >> 1) & 1;
        const int cls = (qc + 2 * h) & 3;  // column residue of the class in this row
        const int c0 = 32 * w;
        // five 64-bit windows, bit b = column c0 - 16 + b (periodic): for L a
        // multiple of 32 the words w - 1, w, w + 1 of the row (modulo nw),
        // else periodic windows built column by column
        uint64_t win[5];
        const int wm = w == 0 ? nw - 1 : w - 1, wp = w + 1 == nw ? 0 : w + 1;
#pragma unroll
        for (int o = 0; o < 5; ++o) {
            int gi = i - 2 + o;
            gi += (gi < 0) ? L : 0;
            gi -= (gi >= L) ? L : 0;
            const uint32_t* row = lat + (size_t)gi * stride;
            uint32_t lo, hi;
            if ((L & 31) == 0) {
                const uint32_t a = row[wm], bw = row[w], c = row[wp];
                lo = funnel(bw, a, 16);
                hi = funnel(c, bw, 16);
            } else if (L >= 32) {
                lo = seg::global_window_wide(row, L, nw, c0 - 16);
                hi = seg::global_window_wide(row, L, nw, c0 + 16);
            } else {
                lo = seg::global_window(row, L, nw, c0 - 16);
                hi = seg::global_window(row, L, nw, c0 + 16);
            }
            win[o] = ((uint64_t)hi << 32) | lo;
            lw[lane * kPdLaneWords + 2 * o] = lo;
            lw[lane * kPdLaneWords + 2 * o + 1] = hi;
        }
        lw[lane * kPdLaneWords + 10] = (uint32_t)i * (uint32_t)L + (uint32_t)c0;
        // columns c0 .. c0 + 31 (bits at columns >= L wrap round in the
        // windows; they are masked off, and the stored word keeps them zero)
        const int valid = min(32, L - c0);
        const uint32_t vmask = valid >= 32 ? 0xFFFFFFFFu : ((1u << valid) - 1u);
        const uint32_t X = (uint32_t)(win[2] >> 16);
        const uint32_t E = (uint32_t)(win[2] >> 17), Wn = (uint32_t)(win[2] >> 15);
        const uint32_t N = (uint32_t)(win[1] >> 16), S = (uint32_t)(win[3] >> 16);
        act = ((X ^ E) | (X ^ Wn) | (X ^ N) | (X ^ S)) & (0x11111111u << cls) & vmask;
        own = X & vmask;
    }
    words[lane] = own;
    // the wave's class sites with a differing neighbour (the others cannot
    // change and draw nothing), compacted into one list: each lane's offset
    // is the exclusive prefix sum of the counts (0..8) below it, taken
    // bit-sliced from four ballots
    const int cnt = __popc(act);
    int pos = 0, total = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const unsigned long long m = __ballot((cnt >> b) & 1);
        pos += seg::lanes_below(m) << b;
        total += __popcll(m) << b;
    }
    while (act) {
        const int bit = __ffs(act) - 1;
        act &= act - 1u;
        list[pos++] = ((uint32_t)lane << 5) | (uint32_t)bit;
    }
    __syncthreads();  // the table, and every wave's windows and list
    // the listed sites, one per lane per pass: Philox block of counter
    // (x, t, k, 0), the neighbour, the two pairwise payoffs, Eq. (3)
    int my_delta = 0;
    for (int qb = 0; qb < total; qb += 64) {
        const int q = qb + lane;
        if (q < total) {
            const uint32_t en = list[q];
            const int sl = (int)(en >> 5), o = (int)(en & 31u);
            const uint32_t* sw = lw + sl * kPdLaneWords;
            uint64_t win[5];
#pragma unroll
            for (int r = 0; r < 5; ++r) win[r] = ((uint64_t)sw[2 * r + 1] << 32) | sw[2 * r];
            const uint4 rnd = philox4x32_10(make_uint4(sw[10] + (uint32_t)o, t, (uint32_t)k, 0u), k0, k1);
            const int d = (int)(rnd.x >> 30);  // 0 E, 1 W, 2 S, 3 N
            const int di = dir_di(d), dj = dir_dj(d);
            const int pc = 16 + o;  // x's column in the windows
            const int sx = (int)bit64(win[2], pc);
            const int sy = (int)bit64(win[2 + di], pc + dj);
            if (sx != sy) {
                const int nx = (int)(bit64(win[1], pc) + bit64(win[3], pc) + bit64(win[2], pc - 1) +
                                     bit64(win[2], pc + 1));
                const int ry = 2 + di, cy = pc + dj;
                const int ny = (int)(bit64(win[ry - 1], cy) + bit64(win[ry + 1], cy) + bit64(win[ry], cy - 1) +
                                     bit64(win[ry], cy + 1));
                const int dir = sx ? 0 : 1;
                if (rnd.y < sT[(dir * 5 + nx) * 5 + ny]) {
                    atomicXor(&words[sl], 1u << o);
                    my_delta += sy ? 1 : -1;
                }
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    const uint32_t out = words[lane];
    if (out != own) lat[(size_t)(p + 2 * ri) * stride + w] = out;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) my_delta += __shfl_xor(my_delta, off, 64);
    if (lane == 0) s_part[wid] = my_delta;
    __syncthreads();
    if (threadIdx.x == 0) {
        int sum = 0;
        for (int q = 0; q < kPdWaves; ++q) sum += s_part[q];
        if (sum) atomicAdd(slot_of(delta, (int)blockIdx.x), (unsigned long long)(long long)sum);
    }
}

hipError_t launch_pd_class(uint32_t* lat, int L, int stride, int k, uint32_t t, uint64_t seed, const uint32_t* T,
                           unsigned long long* delta, hipStream_t st) {
    const int nw = (L + 31) / 32;
    const int64_t tasks = (int64_t)(L / 2) * nw;
    const int blocks = (int)((tasks + kPdThreads - 1) / kPdThreads);
    hipLaunchKernelGGL(k_pd_class, dim3(blocks), dim3(kPdThreads), 0, st, lat, L, stride, nw, k, t, (uint32_t)seed,
                       (uint32_t)(seed >> 32), T, delta);
    return hipGetLastError();
}

}  // namespace pgg
