// Resident sweep for small lattices (gfx950): one workgroup keeps the whole
// periodic lattice in LDS and runs many sweeps per launch.
//
// A small lattice swept one row residue per launch is bound by the launch
// itself (dispatch, window fill, the four class passes' dependency chain,
// about 8 us per residue whatever the size).  Here the lattice's L rows live
// in LDS with three halo rows above and below (copies of the rows across the
// periodic wrap) and one pad word on each side of every row (the word
// across the wrap), so every stencil reads plain LDS offsets.  Per residue a
// the W waves (4, 8 or 16) split the L/4 rows of residue a and run the whole-row update
// of pgg_fullrow.hpp on them (classes 4a..4a+3, lists, flips in place --
// rows of one residue never read each other); a workgroup barrier, the halo
// rows refreshed from the rows they copy, another barrier, the next residue.
// After the last sweep the rows are written back.  For L a multiple of 32,
// 64 <= L <= 512 (the lattice and the wave lists fit the LDS); one CU does the
// work, so other lattices on other streams can use the rest of the device.
// Above L = 256 the lattice and lists need more than 64 KB (104 KB at L =
// 512); gfx950 gives a workgroup up to 160 KB.
// Few waves with many rows each beat many sparse ones: a wave's class pass
// issues about the same instructions whether 8 or 64 of its lanes hold sites,
// and the CU's VALU issue is what bounds the sweep.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pgg_device.hpp"
#include "pgg_fullrow.hpp"
#include "pgg_internal.hpp"
#include "pgg_segment.hpp"

namespace pgg {

namespace {

__host__ __device__ inline int resident_rows_per_wave(int L, int W) { return (L / 4 + W - 1) / W; }
__host__ __device__ inline int resident_list_words(int L, int W) { return resident_rows_per_wave(L, W) * (L / 4) + 8; }

// The resident sweep of one lattice by the calling workgroup of W waves:
// load the lattice into LDS, run n sweeps from t0 (per-sweep count changes
// into delta[q]), write it back.
template <int W>
__device__ __forceinline__ void resident_run(uint32_t* __restrict__ lat, int L, int stride, uint32_t t0, int n,
                                             uint32_t k0, uint32_t k1, const uint32_t* __restrict__ T,
                                             unsigned long long* __restrict__ delta,
                                             unsigned long long* __restrict__ drawn) {
    extern __shared__ uint32_t smem[];
    uint32_t* sT = smem;
    const int nw = L >> 5, ldw = nw + 2;
    // buffer row o holds lattice row o - 3 (periodic): pad word, nw words, pad word
    uint32_t* buf = smem + kSegTableWords;
    const int R = resident_rows_per_wave(L, W);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    uint32_t* list = buf + (L + 6) * ldw + wid * resident_list_words(L, W);
    seg_load_table(sT, T);
    for (int q = threadIdx.x; q < (L + 6) * ldw; q += blockDim.x) {
        const int o = q / ldw;
        int w = q - o * ldw - 1;  // -1 .. nw
        w += (w < 0) ? nw : 0;
        w -= (w >= nw) ? nw : 0;
        int gi = o - 3;  // -3 .. L + 2
        gi += (gi < 0) ? L : 0;
        gi -= (gi >= L) ? L : 0;
        buf[q] = lat[(size_t)gi * stride + w];
    }
    __syncthreads();
    const int r_first = wid * R;
    const int nrows = max(0, min(R, L / 4 - r_first));  // rows of each residue this wave owns
#pragma unroll 1
    for (int q = 0; q < n; ++q) {
        const uint32_t t = t0 + (uint32_t)q;
        int my_delta = 0, my_drawn = 0;
#pragma unroll 1
        for (int a = 0; a < 4; ++a) {
            if (nrows > 0) {
                const int i0 = a + 4 * r_first;  // owned rows i0, i0 + 4, .. (buffer rows i0 + 3, ..)
                fullrow_run(nullptr, L, stride, a, i0, R, nrows, t, k0, k1, sT, buf + i0 * ldw, my_delta, my_drawn,
                            list);
            }
            __syncthreads();
            // halo rows: buffer rows 0..2 copy lattice rows L-3..L-1 (buffer L..L+2),
            // buffer rows L+3..L+5 copy lattice rows 0..2 (buffer 3..5)
            for (int k = threadIdx.x; k < 3 * ldw; k += blockDim.x) {
                buf[k] = buf[L * ldw + k];
                buf[(L + 3) * ldw + k] = buf[3 * ldw + k];
            }
            __syncthreads();
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) my_delta += __shfl_xor(my_delta, off, 64);
        if (lane == 0 && my_delta)
            atomicAdd(slot_of(delta + (size_t)q * kSweepWords, wid), (unsigned long long)(long long)my_delta);
        if (drawn) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) my_drawn += __shfl_xor(my_drawn, off, 64);
            if (lane == 0 && my_drawn) atomicAdd(slot_of(drawn, wid), (unsigned long long)my_drawn);
        }
    }
    for (int q = threadIdx.x; q < L * nw; q += blockDim.x) {
        const int i = q / nw, w = q - i * nw;
        lat[(size_t)i * stride + w] = buf[(i + 3) * ldw + 1 + w];
    }
}

template <int W>
__global__ void __launch_bounds__(64 * W)
k_resident(uint32_t* __restrict__ lat, int L, int stride, uint32_t t0, int n, uint32_t k0, uint32_t k1,
           const uint32_t* __restrict__ T, unsigned long long* __restrict__ delta,
           unsigned long long* __restrict__ drawn) {
    resident_run<W>(lat, L, stride, t0, n, k0, k1, T, delta, drawn);
}

// Ensemble form: workgroup b runs the current chunk (n_active sweeps from
// t0) of replica idx[b], in place, its per-sweep count changes into the
// replica's own counters.
template <int W>
__global__ void __launch_bounds__(64 * W)
k_ens_resident(const EnsRep* __restrict__ reps, const int* __restrict__ idx) {
    const EnsRep& rp = reps[idx[blockIdx.x]];
    if (rp.n_active <= 0) return;
    resident_run<W>(rp.lat, rp.L, rp.stride, rp.t0, rp.n_active, rp.k0, rp.k1, rp.T, rp.delta, rp.drawn);
}

}  // namespace

bool resident_fits(int L) { return L % 32 == 0 && L >= 64 && L <= kResidentMaxL; }
bool resident_waves_valid(int W) { return W == 4 || W == 8 || W == 16; }
int resident_auto_waves(int L) { return L <= 96 ? 4 : 8; }  // 4 to 8 rows of a residue per wave

size_t resident_lds_bytes(int L, int W) {
    const int ldw = L / 32 + 2;
    return ((size_t)kSegTableWords + (size_t)(L + 6) * ldw + (size_t)W * resident_list_words(L, W)) *
           sizeof(uint32_t);
}

hipError_t launch_resident(uint32_t* lat, int L, int stride, int W, uint32_t t0, int n, uint64_t seed,
                           const uint32_t* T, unsigned long long* delta, unsigned long long* drawn, hipStream_t st) {
    if (!resident_fits(L) || !resident_waves_valid(W) || n < 1 || stride < L / 32) return hipErrorInvalidValue;
    const size_t lds = resident_lds_bytes(L, W);
    if (lds > max_dynamic_lds()) return hipErrorInvalidValue;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (W == 4) {
        if (!allow_dynamic_lds((const void*)k_resident<4>, lds)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_resident<4>, dim3(1), dim3(256), lds, st, lat, L, stride, t0, n, k0, k1, T, delta, drawn);
    } else if (W == 8) {
        if (!allow_dynamic_lds((const void*)k_resident<8>, lds)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_resident<8>, dim3(1), dim3(512), lds, st, lat, L, stride, t0, n, k0, k1, T, delta, drawn);
    } else {
        if (!allow_dynamic_lds((const void*)k_resident<16>, lds)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_resident<16>, dim3(1), dim3(1024), lds, st, lat, L, stride, t0, n, k0, k1, T, delta,
                           drawn);
    }
    return hipGetLastError();
}

hipError_t launch_ens_resident(const EnsRep* d_reps, const int* d_idx, int n, int L_max, int W, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (!resident_waves_valid(W)) return hipErrorInvalidValue;
    const size_t lds = resident_lds_bytes(L_max, W);
    if (lds > max_dynamic_lds()) return hipErrorInvalidValue;
    if (W == 4) {
        if (!allow_dynamic_lds((const void*)k_ens_resident<4>, lds)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_ens_resident<4>, dim3(n), dim3(256), lds, st, d_reps, d_idx);
    } else if (W == 8) {
        if (!allow_dynamic_lds((const void*)k_ens_resident<8>, lds)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_ens_resident<8>, dim3(n), dim3(512), lds, st, d_reps, d_idx);
    } else {
        if (!allow_dynamic_lds((const void*)k_ens_resident<16>, lds)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_ens_resident<16>, dim3(n), dim3(1024), lds, st, d_reps, d_idx);
    }
    return hipGetLastError();
}

}  // namespace pgg
