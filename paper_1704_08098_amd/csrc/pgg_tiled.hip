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

__global__ void __launch_bounds__(kTiledThreads)
k_tiled_part(uint32_t* __restrict__ lat, int L, int stride, int part, uint32_t t, uint32_t k0, uint32_t k1,
             const uint32_t* __restrict__ T, unsigned long long* __restrict__ delta) {
    __shared__ uint32_t sT[kTableSize];
    __shared__ uint32_t win[10 * kTiledThreads];  // window row o of lane l at win[o * kTiledThreads + l]
    for (int k = threadIdx.x; k < kTableSize; k += blockDim.x) sT[k] = T[k];
    const int half = L >> 3;  // domains of one type per row of domains
    const int g = (int)blockIdx.x * kTiledThreads + (int)threadIdx.x;
    const bool on = g < half * half;
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
            w[o * kTiledThreads] = seg::global_window(lat + (size_t)gi * stride, L, nw, 4 * J - 3) & 0x3FFu;
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
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) my_delta += __shfl_xor(my_delta, off, 64);
    if ((threadIdx.x & 63) == 0 && my_delta)
        atomicAdd(slot_of(delta, (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6)),
                  (unsigned long long)(long long)my_delta);
}

}  // namespace

hipError_t launch_tiled_part(uint32_t* lat, int L, int stride, int part, uint32_t t, uint64_t seed,
                             const uint32_t* T, unsigned long long* delta, hipStream_t st) {
    if (L % 8 != 0 || part < 0 || part > 3) return hipErrorInvalidValue;
    const int n = (L / 8) * (L / 8);
    const int blocks = (n + kTiledThreads - 1) / kTiledThreads;
    hipLaunchKernelGGL(k_tiled_part, dim3(blocks), dim3(kTiledThreads), 0, st, lat, L, stride, part, t,
                       (uint32_t)seed, (uint32_t)(seed >> 32), T, delta);
    return hipGetLastError();
}

}  // namespace pgg
