// Kernels of the spatial public goods game engine (gfx950).
//
//   fermi_table        Fermi thresholds of Eq. (3) as 32-bit integers (host).
//   k_init_int8/bits   i.i.d. initial strategies (Sec. III) + N_C(0).
//   k_colour_int8      one colour class of the sweep on the int8 layout.
//   k_rowband_bits     the four colour classes of one row residue on the
//                      bit-packed layout, rows staged in LDS.
//   k_count_*, k_pack, k_unpack, k_fill_u64, k_scan_counts: bookkeeping.
#include <hip/hip_runtime.h>

#include <cmath>
#include <stdint.h>

#include "pgg_device.hpp"
#include "pgg_internal.hpp"

namespace pgg {

// ---------------------------------------------------------------------------
// Fermi acceptance table, Sec. III Eq. (3), built once on the host.  With
// c = 1, G = 5 the payoff difference is Pi_x - Pi_y = (r/5) dSigma - 5 ds, so
// the Fermi probability is a function of (dSigma, ds) only;
// T = min(2^32 - 1, floor(W 2^32 + 1/2)).  binary64 with the host's libm exp,
// a fixed operation order and no contraction, so that every table of the
// library (single lattices, ensembles, served jobs) is the same function of
// (r, K) and never depends on a device math library.
// ---------------------------------------------------------------------------
void fermi_table(double r, double K, uint32_t* T) {
#pragma clang fp contract(off)
    for (int idx = 0; idx < kTableSize; ++idx) {
        const int dsig = idx / 3 - 25;  // Sigma_x - Sigma_y
        const int ds = idx % 3 - 1;     // s_x - s_y
        const double dpi = (r * (double)dsig) / 5.0 - 5.0 * (double)ds;
        const double w = 1.0 / (1.0 + std::exp(dpi / K));
        const double scaled = std::floor(w * 4294967296.0 + 0.5);
        T[idx] = scaled >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)scaled;
    }
}

// Threshold on a 32-bit word for "cooperate" in the initial state.
__device__ __forceinline__ uint64_t init_threshold(double p0) {
#pragma clang fp contract(off)
    const double scaled = floor(p0 * 4294967296.0 + 0.5);
    return scaled >= 4294967296.0 ? 4294967296ull : (uint64_t)scaled;
}

__device__ __forceinline__ void block_add_u64(unsigned long long v, unsigned long long* dst) {
    // wave reduction, one atomic per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, v);
}

// ---------------------------------------------------------------------------
// Initial state (Sec. III): s_x = [w0 < P0], Philox counter (x, 0, 0, 1).
// ---------------------------------------------------------------------------
__global__ void k_init_int8(uint8_t* __restrict__ s, int L, double p0, uint32_t k0, uint32_t k1,
                            unsigned long long* __restrict__ nc) {
    const uint64_t P0 = init_threshold(p0);
    const int64_t n = (int64_t)L * L;
    unsigned long long cnt = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x) {
        const uint4 w = philox4x32_10(make_uint4((uint32_t)x, 0u, 0u, 1u), k0, k1);
        const uint8_t v = (uint64_t)w.x < P0 ? 1 : 0;
        s[x] = v;
        cnt += v;
    }
    block_add_u64(cnt, nc);
}

__global__ void k_init_bits(uint32_t* __restrict__ lat, int L, int stride, double p0, uint32_t k0,
                            uint32_t k1, unsigned long long* __restrict__ nc) {
    const uint64_t P0 = init_threshold(p0);
    const int64_t nwords = (int64_t)L * stride;
    unsigned long long cnt = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nwords;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q / stride);
        const int w = (int)(q - (int64_t)i * stride);
        uint32_t word = 0;
        for (int bit = 0; bit < 32; ++bit) {
            const int j = 32 * w + bit;
            if (j >= L) break;
            const uint32_t x = (uint32_t)i * (uint32_t)L + (uint32_t)j;
            const uint4 r = philox4x32_10(make_uint4(x, 0u, 0u, 1u), k0, k1);
            word |= ((uint64_t)r.x < P0 ? 1u : 0u) << bit;
        }
        lat[q] = word;
        cnt += __popc(word);
    }
    block_add_u64(cnt, nc);
}

// ---------------------------------------------------------------------------
// Reference sweep on the int8 layout: one launch per colour class k = 4a + b.
// Thread -> site (i, j) = (a + 4I, b + 4J).  Every site of the class draws
// its Philox block, picks y, and (if the strategies differ) compares the
// acceptance word with the threshold of (Sigma_x - Sigma_y, s_x - s_y).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int sigma_int8(const uint8_t* __restrict__ s, int L, int i, int j) {
    const int im1 = wrap_add(i, -1, L), ip1 = wrap_add(i, 1, L);
    const int im2 = wrap_add(i, -2, L), ip2 = wrap_add(i, 2, L);
    const int jm1 = wrap_add(j, -1, L), jp1 = wrap_add(j, 1, L);
    const int jm2 = wrap_add(j, -2, L), jp2 = wrap_add(j, 2, L);
    const uint8_t* r0 = s + (size_t)i * L;
    const uint8_t* rm1 = s + (size_t)im1 * L;
    const uint8_t* rp1 = s + (size_t)ip1 * L;
    const int centre = r0[j];
    const int near = r0[jm1] + r0[jp1] + rm1[j] + rp1[j];
    const int diag = rm1[jm1] + rm1[jp1] + rp1[jm1] + rp1[jp1];
    const int far = r0[jm2] + r0[jp2] + s[(size_t)im2 * L + j] + s[(size_t)ip2 * L + j];
    return 5 * centre + 2 * near + 2 * diag + far;
}

__global__ void __launch_bounds__(256)
k_colour_int8(uint8_t* __restrict__ s, int L, int a, int b, uint32_t t, uint32_t k0, uint32_t k1,
              const uint32_t* __restrict__ T, unsigned long long* __restrict__ delta) {
    __shared__ uint32_t sT[kTableSize];
    for (int q = threadIdx.x; q < kTableSize; q += blockDim.x) sT[q] = T[q];
    __syncthreads();
    const int n = L >> 2;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    int change = 0;
    if (idx < n * n) {
        const int I = idx / n, J = idx - (idx / n) * n;
        const int i = a + 4 * I, j = b + 4 * J;
        const uint32_t k = (uint32_t)(4 * a + b);
        const uint4 w = philox4x32_10(make_uint4((uint32_t)(i * L + j), t, k, 0u), k0, k1);
        const int d = (int)(w.x >> 30);
        const uint32_t u = w.y;
        const int yi = wrap_add(i, dir_di(d), L), yj = wrap_add(j, dir_dj(d), L);
        const int sx = s[(size_t)i * L + j], sy = s[(size_t)yi * L + yj];
        if (sx != sy) {
            const int dsig = sigma_int8(s, L, i, j) - sigma_int8(s, L, yi, yj);
            if (u < sT[(dsig + 25) * 3 + (sx - sy + 1)]) {
                s[(size_t)i * L + j] = (uint8_t)sy;
                change = sy ? 1 : -1;
            }
        }
    }
    const long long up = __popcll(__ballot(change > 0));
    const long long dn = __popcll(__ballot(change < 0));
    if ((threadIdx.x & 63) == 0 && up != dn)
        atomicAdd(slot_of(delta, (int)(blockIdx.x * 4 + (threadIdx.x >> 6))), (unsigned long long)(up - dn));
}

// ---------------------------------------------------------------------------
// Bit-packed sweep: one launch per row residue a = i mod 4 runs the four
// colour classes k = 4a + 0..3.  Within those four classes a site at row i
// reads rows i-3..i+3 but only sites of its own row change (the other rows
// of the residue are 4 or more rows away), so a workgroup owning R rows of
// the residue stages rows i0-3 .. i0+4(R-1)+3 in LDS, runs the four classes
// with a barrier between them, and writes its R rows back.  Workgroups of
// one launch never read each other's rows.
//
// COMPACT: before each class, the sites whose four neighbours all share
// their strategy are dropped (copying an equal strategy is a no-op, and the
// counter-based generator needs no draw to stay in step); the remaining
// sites are appended to an LDS list and processed densely.
// ---------------------------------------------------------------------------
template <bool COMPACT>
__global__ void __launch_bounds__(kRowbandThreads)
k_rowband_bits(uint32_t* __restrict__ lat, int L, int stride, int nw, int a, int R, uint32_t t,
               uint32_t k0, uint32_t k1, const uint32_t* __restrict__ T,
               unsigned long long* __restrict__ delta, unsigned long long* __restrict__ drawn) {
    extern __shared__ uint32_t smem[];
    const int ldw = nw + 1;             // one zero pad word per staged row
    const int rows = 4 * R + 3;
    uint32_t* sT = smem;                // kTableSize words (padded to 160)
    uint32_t* img = smem + 160;         // rows * ldw words
    uint32_t* list = img + rows * ldw;  // COMPACT: R * L/4 entries
    __shared__ int s_count[4];
    __shared__ int s_delta;

    const int q4 = L >> 2;              // sites per row per colour class
    const int g = blockIdx.x;
    const int i0 = a + 4 * R * g;       // first owned row
    const int Rv = min(R, q4 - g * R);  // owned rows in this band

    for (int q = threadIdx.x; q < kTableSize; q += blockDim.x) sT[q] = T[q];
    if (threadIdx.x < 4) s_count[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_delta = 0;
    const int nrows = 4 * Rv + 3;
    for (int q = threadIdx.x; q < nrows * ldw; q += blockDim.x) {
        const int rho = q / ldw, w = q - (q / ldw) * ldw;
        int gi = i0 - 3 + rho;
        gi += (gi < 0) ? L : 0;
        gi -= (gi >= L) ? L : 0;
        img[q] = (w < nw) ? lat[(size_t)gi * stride + w] : 0u;
    }
    __syncthreads();

    int my_delta = 0;
    for (int b = 0; b < 4; ++b) {
        const uint32_t k = (uint32_t)(4 * a + b);
        int n_items;
        if (COMPACT) {
            const uint32_t colmask = 0x11111111u << b;
            for (int q = threadIdx.x; q < Rv * nw; q += blockDim.x) {
                const int m = q / nw, w = q - (q / nw) * nw;
                const uint32_t* r0 = img + (3 + 4 * m) * ldw;
                const uint32_t X = r0[w];
                const uint32_t N = r0[w - ldw];
                const uint32_t S = r0[w + ldw];
                const uint32_t E = row_window(r0, L, 32 * w + 1);
                const uint32_t Wn = row_window(r0, L, 32 * w - 1);
                const int valid = L - 32 * w;
                const uint32_t vmask = valid >= 32 ? 0xFFFFFFFFu : ((1u << valid) - 1u);
                uint32_t act = ((X ^ E) | (X ^ Wn) | (X ^ N) | (X ^ S)) & colmask & vmask;
                const int cnt = __popc(act);
                if (cnt) {
                    int pos = atomicAdd(&s_count[b], cnt);
                    while (act) {
                        const int bit = __ffs(act) - 1;
                        act &= act - 1u;
                        list[pos++] = ((uint32_t)m << 16) | (uint32_t)(32 * w + bit);
                    }
                }
            }
            __syncthreads();
            n_items = s_count[b];
        } else {
            n_items = Rv * q4;
        }
        for (int e = threadIdx.x; e < n_items; e += blockDim.x) {
            int m, j;
            if (COMPACT) {
                const uint32_t ent = list[e];
                m = (int)(ent >> 16);
                j = (int)(ent & 0xFFFFu);
            } else {
                m = e / q4;
                j = b + 4 * (e - m * q4);
            }
            uint32_t* r0 = img + (3 + 4 * m) * ldw;
            const int c = j - 16;
            const uint32_t wm3 = row_window(r0 - 3 * ldw, L, c);
            const uint32_t wm2 = row_window(r0 - 2 * ldw, L, c);
            const uint32_t wm1 = row_window(r0 - ldw, L, c);
            const uint32_t w00 = row_window(r0, L, c);
            const uint32_t wp1 = row_window(r0 + ldw, L, c);
            const uint32_t wp2 = row_window(r0 + 2 * ldw, L, c);
            const uint32_t wp3 = row_window(r0 + 3 * ldw, L, c);
            const int i = i0 + 4 * m;
            const uint4 rnd = philox4x32_10(make_uint4((uint32_t)(i * L + j), t, k, 0u), k0, k1);
            const int d = (int)(rnd.x >> 30);
            const uint32_t u = rnd.y;
            const int o = dir_di(d);          // row offset of y
            const int p = 16 + dir_dj(d);     // bit of y's column in the windows
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

    for (int q = threadIdx.x; q < Rv * nw; q += blockDim.x) {
        const int m = q / nw, w = q - (q / nw) * nw;
        lat[(size_t)(i0 + 4 * m) * stride + w] = img[(3 + 4 * m) * ldw + w];
    }
    if (my_delta) atomicAdd(&s_delta, my_delta);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_delta) atomicAdd(slot_of(delta, (int)blockIdx.x), (unsigned long long)(long long)s_delta);
        if (drawn) {  // diagnostics: number of site updates that drew random numbers
            const int n = COMPACT ? s_count[0] + s_count[1] + s_count[2] + s_count[3] : 4 * Rv * q4;
            atomicAdd(slot_of(drawn, (int)blockIdx.x), (unsigned long long)n);
        }
    }
}

// ---------------------------------------------------------------------------
// Bookkeeping kernels.
// ---------------------------------------------------------------------------
__global__ void k_count_int8(const uint8_t* __restrict__ s, int64_t n, unsigned long long* nc) {
    unsigned long long cnt = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (int64_t)gridDim.x * blockDim.x)
        cnt += s[x];
    block_add_u64(cnt, nc);
}

__global__ void k_count_bits(const uint32_t* __restrict__ lat, int64_t nwords, unsigned long long* nc) {
    unsigned long long cnt = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nwords;
         q += (int64_t)gridDim.x * blockDim.x)
        cnt += __popc(lat[q]);
    block_add_u64(cnt, nc);
}

// int8 (0/1 bytes) -> bit-packed rows; padding bits and words are zero.  One
// thread per word, reading its 32 bytes as 4-byte groups (L is a multiple of
// 4, so a group never crosses a row end and row starts are 4-byte aligned).
__device__ __forceinline__ uint32_t nibble_of_bytes(uint32_t v) {
    v &= 0x01010101u;
    return (v | (v >> 7) | (v >> 14) | (v >> 21)) & 0xFu;
}

__global__ void k_pack(const uint8_t* __restrict__ s, uint32_t* __restrict__ lat, int L, int stride) {
    const int64_t nwords = (int64_t)L * stride;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nwords;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(q / stride), w = (int)(q - (q / stride) * stride);
        const uint32_t* row = (const uint32_t*)(s + (size_t)i * L);
        uint32_t word = 0;
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            const int j = 32 * w + 4 * g;
            if (j < L) word |= nibble_of_bytes(row[j >> 2]) << (4 * g);
        }
        lat[q] = word;
    }
}

// Bit-packed rows -> int8 bytes, one thread per 4 bytes of a row.
__global__ void k_unpack(const uint32_t* __restrict__ lat, uint8_t* __restrict__ s, int L, int stride) {
    const int64_t n4 = (int64_t)L * (L / 4);
    const int q4 = L / 4;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n4;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(x / q4), j = 4 * (int)(x - (x / q4) * q4);
        const uint32_t b = (lat[(size_t)i * stride + (j >> 5)] >> (j & 31)) & 0xFu;
        ((uint32_t*)s)[x] = (b & 1u) | ((b & 2u) << 7) | ((b & 4u) << 14) | ((b & 8u) << 21);
    }
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int64_t n, unsigned long long v) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        p[q] = v;
}

// counts[q] = nc + sum_{q' <= q} (sum of the kSlots slots of sweep q') in
// two's complement, then nc = counts[n - 1].  One block of 1024 threads;
// each owns a contiguous chunk of sweeps.
__device__ __forceinline__ unsigned long long sweep_delta(const unsigned long long* __restrict__ delta, int q) {
    unsigned long long v = 0;
    const unsigned long long* row = delta + (size_t)q * kSweepWords;
#pragma unroll 8
    for (int k = 0; k < kSlots; ++k) v += row[k * kSlotStride];
    return v;
}

__global__ void __launch_bounds__(1024)
k_scan_counts(const unsigned long long* __restrict__ delta, unsigned long long* __restrict__ counts,
              int n, unsigned long long* __restrict__ nc) {
    __shared__ unsigned long long part[1024];
    const int tid = threadIdx.x;
    const int chunk = (n + 1023) / 1024;
    const int lo = min(n, tid * chunk), hi = min(n, lo + chunk);
    unsigned long long sum = 0;
    for (int q = lo; q < hi; ++q) sum += sweep_delta(delta, q);
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const unsigned long long v = tid >= off ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    unsigned long long run = *nc + (tid ? part[tid - 1] : 0ull);
    for (int q = lo; q < hi; ++q) {
        run += sweep_delta(delta, q);
        counts[q] = run;
    }
    __syncthreads();
    if (tid == 1023) *nc = *nc + part[1023];
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
static int grid_for(int64_t n, int block, int cap = 65536) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t upload_table(const uint32_t* host_T, uint32_t* T, hipStream_t st) {
    return hipMemcpyAsync(T, host_T, kTableSize * sizeof(uint32_t), hipMemcpyHostToDevice, st);
}

hipError_t launch_init(int layout, void* lat, int L, int stride, double p0, uint64_t seed,
                       unsigned long long* nc, hipStream_t st) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, nc, (int64_t)1, 0ull);
    if (layout == 0) {
        const int64_t n = (int64_t)L * L;
        hipLaunchKernelGGL(k_init_int8, dim3(grid_for(n, 256)), dim3(256), 0, st, (uint8_t*)lat, L,
                           p0, k0, k1, nc);
    } else {
        const int64_t n = (int64_t)L * stride;
        hipLaunchKernelGGL(k_init_bits, dim3(grid_for(n, 256)), dim3(256), 0, st, (uint32_t*)lat, L,
                           stride, p0, k0, k1, nc);
    }
    return hipGetLastError();
}

hipError_t launch_count(int layout, const void* lat, int L, int stride, unsigned long long* nc,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, nc, (int64_t)1, 0ull);
    if (layout == 0) {
        const int64_t n = (int64_t)L * L;
        hipLaunchKernelGGL(k_count_int8, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st,
                           (const uint8_t*)lat, n, nc);
    } else {
        const int64_t n = (int64_t)L * stride;
        hipLaunchKernelGGL(k_count_bits, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st,
                           (const uint32_t*)lat, n, nc);
    }
    return hipGetLastError();
}

hipError_t launch_pack(const uint8_t* s, uint32_t* lat, int L, int stride, hipStream_t st) {
    hipLaunchKernelGGL(k_pack, dim3(grid_for((int64_t)L * stride, 256)), dim3(256), 0, st, s, lat, L,
                       stride);
    return hipGetLastError();
}

hipError_t launch_unpack(const uint32_t* lat, uint8_t* s, int L, int stride, hipStream_t st) {
    hipLaunchKernelGGL(k_unpack, dim3(grid_for((int64_t)L * (L / 4), 256)), dim3(256), 0, st, lat, s, L,
                       stride);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_scan_counts(const unsigned long long* delta, unsigned long long* counts, int n,
                              unsigned long long* nc, hipStream_t st) {
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, delta, counts, n, nc);
    return hipGetLastError();
}

hipError_t launch_colour_phase(uint8_t* s, int L, int k, uint32_t t, uint64_t seed,
                               const uint32_t* T, unsigned long long* delta, hipStream_t st) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int64_t per = (int64_t)(L / 4) * (L / 4);
    const int grid = (int)((per + 255) / 256);
    hipLaunchKernelGGL(k_colour_int8, dim3(grid), dim3(256), 0, st, s, L, k / 4, k % 4, t, k0, k1, T,
                       delta);
    return hipGetLastError();
}

size_t rowband_lds_bytes(int L, int R, bool compact) {
    const int nw = (L + 31) / 32;
    size_t words = 160 + (size_t)(4 * R + 3) * (nw + 1);
    if (compact) words += (size_t)R * (L / 4);
    return words * sizeof(uint32_t);
}

hipError_t launch_rowband_residue(uint32_t* lat, int L, int stride, int R, bool compact, int a,
                                  uint32_t t, uint64_t seed, const uint32_t* T,
                                  unsigned long long* delta, unsigned long long* drawn,
                                  hipStream_t st) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int nw = (L + 31) / 32;
    const int bands = (L / 4 + R - 1) / R;
    const size_t lds = rowband_lds_bytes(L, R, compact);
    if (!allow_dynamic_lds(compact ? (const void*)k_rowband_bits<true> : (const void*)k_rowband_bits<false>, lds))
        return hipErrorInvalidValue;
    if (compact)
        hipLaunchKernelGGL(k_rowband_bits<true>, dim3(bands), dim3(kRowbandThreads), lds, st, lat, L,
                           stride, nw, a, R, t, k0, k1, T, delta, drawn);
    else
        hipLaunchKernelGGL(k_rowband_bits<false>, dim3(bands), dim3(kRowbandThreads), lds, st, lat, L,
                           stride, nw, a, R, t, k0, k1, T, delta, drawn);
    return hipGetLastError();
}

}  // namespace pgg
