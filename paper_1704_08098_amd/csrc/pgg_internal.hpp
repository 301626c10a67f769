// Host-side launchers of the engine's kernels (implemented in pgg_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pgg {

constexpr int kTableSize = 153;       // 51 values of dSigma x 3 values of ds
constexpr int kRowbandThreads = 256;  // workgroup size of the row-band kernel

hipError_t launch_build_table(double r, double K, uint32_t* T, hipStream_t st);
hipError_t launch_init(int layout, void* lat, int L, int stride, double p0, uint64_t seed,
                       unsigned long long* nc, hipStream_t st);
hipError_t launch_count(int layout, const void* lat, int L, int stride, unsigned long long* nc,
                        hipStream_t st);
hipError_t launch_pack(const uint8_t* s, uint32_t* lat, int L, int stride, hipStream_t st);
hipError_t launch_unpack(const uint32_t* lat, uint8_t* s, int L, int stride, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st);
hipError_t launch_scan_counts(const unsigned long long* delta, unsigned long long* counts, int n,
                              unsigned long long* nc, hipStream_t st);
// One colour class k of sweep t on the int8 layout (16 per sweep), adding
// the net change of the cooperator count to *delta.
hipError_t launch_colour_phase(uint8_t* s, int L, int k, uint32_t t, uint64_t seed,
                               const uint32_t* T, unsigned long long* delta, hipStream_t st);
// The four colour classes of row residue a of sweep t on the bits layout
// (4 per sweep).  drawn (optional) counts updates that drew random numbers.
hipError_t launch_rowband_residue(uint32_t* lat, int L, int stride, int R, bool compact, int a,
                                  uint32_t t, uint64_t seed, const uint32_t* T,
                                  unsigned long long* delta, unsigned long long* drawn,
                                  hipStream_t st);
size_t rowband_lds_bytes(int L, int R, bool compact);
// Staged variant (pgg_staged.hip): all four classes draw in one batch.
hipError_t launch_staged_residue(uint32_t* lat, int L, int stride, int R, int a, uint32_t t,
                                 uint64_t seed, const uint32_t* T, unsigned long long* delta,
                                 unsigned long long* drawn, hipStream_t st);
size_t staged_lds_bytes(int L, int R);
constexpr size_t kMaxDynamicLds = 64 * 1024;

}  // namespace pgg
