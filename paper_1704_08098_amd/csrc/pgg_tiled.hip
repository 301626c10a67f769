// The double tiling decomposition of Sec. IV (Fig. 2) on the bit-packed
// layout: the paper's own parallel dynamics, as a second schedule beside the
// 16-colour sweep.
//
// The lattice is cut into 4 x 4 domains (I, J) (rows 4I..4I+3, columns
// 4J..4J+3) of four types, type 1 + 2 (I mod 2) + (J mod 2).  A Monte Carlo
// step is four launches, one per type; in its launch every domain of the
// type takes 16 elementary steps (Sec. III) in random sequential order: the
// player x is drawn uniformly among the domain's 16 and its neighbour y
// uniformly among x's four, so y may lie outside the domain.  Random
// numbers: step m of part p in sweep t of domain (I, J) takes the Philox
// block of counter (I L/4 + J, t, 16 p + m, 2); x = player w0 >> 28 of the
// domain (row-major), d = (w0 >> 26) mod 4 (E, W, S, N), u = w1.
//
// One lane per domain.  A step reads at most 3 sites beyond its domain (the
// groups of x and of y), so the lane copies the 10 x 10 block of rows
// 4I-3..4I+6 and columns 4J-3..4J+6 into LDS (one 32-bit word per row,
// bits 0..9), runs its 16 steps there, and writes back the changed bits of
// its 4 x 4 domain.  Domains of one type are 4 sites apart, so no lane reads
// a site another lane of the launch writes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pgg_device.hpp"
#include "pgg_internal.hpp"
#include "pgg_segment.hpp"

namespace pgg {

namespace {

constexpr int kTiledThreads = 256;

// The sigma stencil at window column c of window rows r-2 .. r+2 (c in
// [2, 7]): the rows shifted so that column c sits at bit 16.
__device__ __forceinline__ int tiled_rest(const uint32_t* __restrict__ w, int r, int c) {
    const int sh = 16 - c;
    return seg::sigma_rest16(w[(r - 2) * kTiledThreads] << sh, w[(r - 1) * kTiledThreads] << sh,
                             w[r * kTiledThreads] << sh, w[(r + 1) * kTiledThreads] << sh,
                             w[(r + 2) * kTiledThreads] << sh);
}

// The 16 random sequential steps of the domain of lane g (0 <= g <
// (L/8)^2, or on == false for a padding lane) of part `part` in sweep t:
// fill the lane's window, run the steps, write back the changed bits.  sT:
// the threshold table in LDS (loaded and synchronised by the caller before
// this is called; the function synchronises the workgroup once itself).
// Returns the net change of the cooperator count.
__device__ __forceinline__ int tiled_domain(uint32_t* __restrict__ lat, int L, int stride, int part, uint32_t t,
                                            uint32_t k0, uint32_t k1, const uint32_t* __restrict__ sT,
                                            uint32_t* __restrict__ win, int g, bool on) {
    const int half = L >> 3;  // domains of one type per row of domains
    const int I = (part >> 1) + 2 * (on ? g / half : 0);
    const int J = (part & 1) + 2 * (on ? g % half : 0);
    const int nw = (L + 31) >> 5;
    uint32_t* w = win + threadIdx.x;
    uint32_t orig[4] = {0u, 0u, 0u, 0u};
    if (on) {
        for (int o = 0; o < 10; ++o) {
            int gi = 4 * I - 3 + o;  // in [-3, L + 6)
            gi += (gi < 0) ? L : 0;
            gi -= (gi >= L) ? L : 0;
            const uint32_t* row = lat + (size_t)gi * stride;
            const uint32_t bits = L >= 32 ? seg::global_window_wide(row, L, nw, 4 * J - 3)
                                          : seg::global_window(row, L, nw, 4 * J - 3);
            w[o * kTiledThreads] = bits & 0x3FFu;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) orig[q] = (w[(3 + q) * kTiledThreads] >> 3) & 0xFu;
    }
    __syncthreads();
    int my_delta = 0;
    if (on) {
        const uint32_t D = (uint32_t)(I * (L >> 2) + J);
        // The random words do not depend on the lattice: draw all 16 first
        // (independent Philox blocks, so they overlap), then run the steps,
        // whose chain is only the LDS stencil and the flip.
        uint2 rnd[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) rnd[m] = philox4x32_10_w01(D, t, (uint32_t)(16 * part + m), 2u, k0, k1);
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int idx = (int)(rnd[m].x >> 28);
            const int d = (int)((rnd[m].x >> 26) & 3u);
            const int rx = 3 + (idx >> 2), cx = 3 + (idx & 3);  // window position of x
            const int ry = rx + dir_di(d), cy = cx + dir_dj(d);
            const int sx = (int)((w[rx * kTiledThreads] >> cx) & 1u);
            const int sy = (int)((w[ry * kTiledThreads] >> cy) & 1u);
            const int ds = sx - sy;
            if (ds != 0) {  // copying an equal strategy changes nothing
                const int dsig = tiled_rest(w, rx, cx) - tiled_rest(w, ry, cy) + 5 * ds;
                if (rnd[m].y < sT[(dsig + 25) * 3 + ds + 1]) {
                    w[rx * kTiledThreads] ^= 1u << cx;
                    my_delta += sy ? 1 : -1;
                }
            }
        }
        // write back the domain's changed bits (other lanes write other
        // nibbles of the same words, hence the atomic XOR)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t diff = ((w[(3 + q) * kTiledThreads] >> 3) & 0xFu) ^ orig[q];
            if (diff) {
                const int col = 4 * J;
                atomicXor(lat + (size_t)(4 * I + q) * stride + (col >> 5), diff << (col & 31));
            }
        }
    }
    return my_delta;
}

__device__ __forceinline__ void add_delta(int my_delta, unsigned long long* __restrict__ delta) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) my_delta += __shfl_xor(my_delta, off, 64);
    if ((threadIdx.x & 63) == 0 && my_delta)
        atomicAdd(slot_of(delta, (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6)),
                  (unsigned long long)(long long)my_delta);
}

__global__ void __launch_bounds__(kTiledThreads)
k_tiled_part(uint32_t* __restrict__ lat, int L, int stride, int part, uint32_t t, uint32_t k0, uint32_t k1,
             const uint32_t* __restrict__ T, unsigned long long* __restrict__ delta) {
    __shared__ uint32_t sT[kTableSize];
    __shared__ uint32_t win[10 * kTiledThreads];  // window row o of lane l at win[o * kTiledThreads + l]
    for (int k = threadIdx.x; k < kTableSize; k += blockDim.x) sT[k] = T[k];
    const int g = (int)blockIdx.x * kTiledThreads + (int)threadIdx.x;
    const int my_delta = tiled_domain(lat, L, stride, part, t, k0, k1, sT, win, g, g < (L >> 3) * (L >> 3));
    add_delta(my_delta, delta);
}

// Replica whose workgroup range holds workgroup b: the last with wave_base <= b.
__device__ __forceinline__ int replica_of_block(const EnsRep* __restrict__ reps, int n, int b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (reps[mid].wave_base <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// One part of sweep q of a chunk for every replica of a tiled ensemble: the
// workgroups are dealt out replica by replica (wave_base = first workgroup),
// and each replica updates in place.
__global__ void __launch_bounds__(kTiledThreads)
k_ens_tiled_part(const EnsRep* __restrict__ reps, int n_reps, int part, int q) {
    __shared__ uint32_t sT[kTableSize];
    __shared__ uint32_t win[10 * kTiledThreads];
    const int rep_id = __builtin_amdgcn_readfirstlane(replica_of_block(reps, n_reps, (int)blockIdx.x));
    const EnsRep& rp = reps[rep_id];
    for (int k = threadIdx.x; k < kTableSize; k += blockDim.x) sT[k] = rp.T[k];
    const int L = rp.L;
    const int g = ((int)blockIdx.x - rp.wave_base) * kTiledThreads + (int)threadIdx.x;
    const bool on = q < rp.n_active && g < (L >> 3) * (L >> 3);
    const int my_delta = tiled_domain(rp.lat, L, rp.stride, part, rp.t0 + (uint32_t)q, rp.k0, rp.k1, sT, win, g, on);
    add_delta(my_delta, rp.delta + (size_t)q * kSweepWords);
}

}  // namespace

int tiled_blocks(int L) {
    const int n = (L / 8) * (L / 8);
    return (n + kTiledThreads - 1) / kTiledThreads;
}

hipError_t launch_tiled_part(uint32_t* lat, int L, int stride, int part, uint32_t t, uint64_t seed,
                             const uint32_t* T, unsigned long long* delta, hipStream_t st) {
    if (L % 8 != 0 || part < 0 || part > 3) return hipErrorInvalidValue;
    const int blocks = tiled_blocks(L);
    hipLaunchKernelGGL(k_tiled_part, dim3(blocks), dim3(kTiledThreads), 0, st, lat, L, stride, part, t,
                       (uint32_t)seed, (uint32_t)(seed >> 32), T, delta);
    return hipGetLastError();
}

hipError_t launch_ens_tiled_chunk(EnsRep* d_reps, int n, int total_blocks, int len, int chunk,
                                  unsigned long long* counts, hipStream_t st) {
    hipError_t err = launch_ens_begin(d_reps, n, len, chunk, true, st);
    for (int q = 0; err == hipSuccess && q < len; ++q)
        for (int part = 0; err == hipSuccess && part < 4; ++part) {
            hipLaunchKernelGGL(k_ens_tiled_part, dim3(total_blocks), dim3(kTiledThreads), 0, st, d_reps, n, part, q);
            err = hipGetLastError();
        }
    if (err != hipSuccess) return err;
    return launch_ens_end(d_reps, n, chunk, counts, st);
}

}  // namespace pgg
