// Host-side launchers of the engine's kernels (implemented in pgg_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pgg {

constexpr int kTableSize = 153;       // 51 values of dSigma x 3 values of ds
constexpr int kRowbandThreads = 256;  // workgroup size of the row-band kernels

// Per-sweep counters (net change of the cooperator count, draws) are spread
// over kSlots addresses kSlotStride words apart (one 128-byte line each):
// thousands of workgroups adding to one address from 8 XCDs serialise.
constexpr int kSlots = 32;
constexpr int kSlotStride = 16;
constexpr int kSweepWords = kSlots * kSlotStride;  // 64-bit words per sweep
__device__ __forceinline__ unsigned long long* slot_of(unsigned long long* base, int id) {
    return base + (id & (kSlots - 1)) * kSlotStride;
}

// The kTableSize Fermi thresholds T[(dSigma + 25) * 3 + ds + 1] of (r, K),
// computed on the host (binary64), and their upload to a device table.  The
// host array must stay valid until the copy has completed on st.
void fermi_table(double r, double K, uint32_t* host_T);
hipError_t upload_table(const uint32_t* host_T, uint32_t* T, hipStream_t st);
hipError_t launch_init(int layout, void* lat, int L, int stride, double p0, uint64_t seed,
                       unsigned long long* nc, hipStream_t st);
hipError_t launch_count(int layout, const void* lat, int L, int stride, unsigned long long* nc,
                        hipStream_t st);
hipError_t launch_pack(const uint8_t* s, uint32_t* lat, int L, int stride, hipStream_t st);
hipError_t launch_unpack(const uint32_t* lat, uint8_t* s, int L, int stride, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t st);
hipError_t launch_scan_counts(const unsigned long long* delta, unsigned long long* counts, int n,
                              unsigned long long* nc, hipStream_t st);
// Every launcher below takes `delta`, the kSweepWords counters of one sweep
// (the net change of the cooperator count is added to one of its slots), and
// an optional `drawn` of kSweepWords counters for the number of updates that
// drew random numbers.
// One colour class k of sweep t on the int8 layout (16 per sweep).
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
// Double tiling (pgg_tiled.hip): part p (domain type 1 + p) of sweep t, every
// domain of that type taking its 16 random sequential steps (4 per sweep).
// L must be a multiple of 8.
hipError_t launch_tiled_part(uint32_t* lat, int L, int stride, int part, uint32_t t, uint64_t seed,
                             const uint32_t* T, unsigned long long* delta, hipStream_t st);
// Workgroups of one tiled launch for side L.
int tiled_blocks(int L);
// The pairwise prisoner's dilemma (pgg_pd.hip): the 50 thresholds
// T[(dir * 5 + n_x) * 5 + n_y] for temptation b and noise K (host, binary64),
// and one class k (0..7) of sweep t of the 8-colour schedule on the bits
// layout, in place.
constexpr int kPdTableSize = 50;
void pd_table(double b, double K, uint32_t* host_T);
hipError_t launch_pd_class(uint32_t* lat, int L, int stride, int k, uint32_t t, uint64_t seed, const uint32_t* T,
                           unsigned long long* delta, hipStream_t st);
// Resident sweep (pgg_resident.hip): one workgroup of W waves (4, 8 or 16)
// holds the lattice in LDS and runs n sweeps from sweep index t0; delta[q]
// (kSweepWords each) receives sweep t0 + q.  L a multiple of 32, 64 <= L <= 512
// (104 KB of LDS at L = 512).
bool resident_fits(int L);
bool resident_waves_valid(int W);
int resident_auto_waves(int L);
size_t resident_lds_bytes(int L, int W);
hipError_t launch_resident(uint32_t* lat, int L, int stride, int W, uint32_t t0, int n, uint64_t seed,
                           const uint32_t* T, unsigned long long* delta, unsigned long long* drawn, hipStream_t st);
constexpr int kResidentMaxL = 512;
// LDS one workgroup may allocate on the current device
// (hipDeviceAttributeMaxSharedMemoryPerBlock: 160 KB on gfx950; 64 KB if the
// query fails), looked up once per device.
size_t max_dynamic_lds();
// Lets `kernel` be launched with `bytes` of dynamic LDS (the per-kernel
// attribute, set only above 64 KB); false if the runtime refuses.
bool allow_dynamic_lds(const void* kernel, size_t bytes);

// Persistent strip kernel (pgg_strip.hip).  One task per workgroup: rows
// [r0, r0 + H) of one lattice, the tasks owning the strips above (up) and
// below (down) -- the task itself when the strip is the whole lattice --,
// and n sweeps starting at sweep index t0.  delta[q] receives the net change
// of the cooperator count in sweep t0 + q; drawn (optional) counts the
// updates that drew random numbers.
constexpr int kStripThreads = 512;
struct StripTask {
    uint32_t* lat;
    const uint32_t* T;
    unsigned long long* delta;
    unsigned long long* drawn;
    int L, stride, nw, r0, H, up, down, n;
    uint32_t t0, k0, k1, pad;
};
hipError_t launch_strip(const StripTask* d_tasks, int n_tasks, uint64_t* ring, uint32_t* abort_flag,
                        uint64_t wait_ticks, int G, size_t lds, hipStream_t st);
size_t strip_lds_bytes(int L, int H, int G);
hipError_t strip_capacity(size_t lds, int* blocks_per_cu, int* cus);
// Set t0, n and delta of every task (single-lattice runs).
hipError_t launch_tasks_set(StripTask* tasks, int n_tasks, uint32_t t0, int n,
                            unsigned long long* delta, unsigned long long* drawn, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);

// Segment kernel (pgg_segment.hpp, launched by pgg_ensemble.hip): one wave
// per row segment.  Out of place within a sweep: launch a reads residues < a
// from the buffer it writes and the rest from the other one; after the 4
// launches of a sweep the written buffer holds the whole lattice.
constexpr int kWavesPerGroup = 4;  // default waves (segments) per workgroup; 2, 4 or 8

// Ensemble replica descriptor (pgg_ensemble.hip): replica lattice, its
// threshold table, its per-sweep counters (chunk x kSweepWords), geometry,
// the first wave of its range in a launch, the number of sweeps of the
// current chunk, Philox key and current sweep index.
struct EnsRep {
    uint32_t* lat;              // the lattice at chunk boundaries
    uint32_t* lat2;             // second buffer: odd sweeps of a chunk land here
    const uint32_t* T;
    unsigned long long* delta;  // chunk x kSweepWords
    unsigned long long* nc;     // N_C after the last completed sweep
    unsigned long long* drawn;  // kSweepWords spread counters of draws, or null
    int L, stride, nw, segw, nseg, wave_base, n_active;
    int rpw;                    // full-row sweep (segw == L): rows per wave; 0 = segments
    uint32_t k0, k1, t0;
    int tiled;                  // 1: the double-tiling schedule (in place; wave_base counts workgroups)
    int resident;               // 1: swept by the resident kernel (in place, a chunk per launch; no segment waves)
};

// Ensemble form of the resident sweep: workgroup b of n runs the current
// chunk of replica d_idx[b] (n_active sweeps from t0, in place); L_max is
// the largest side among them (it sizes the LDS), W waves per workgroup.
hipError_t launch_ens_resident(const EnsRep* d_reps, const int* d_idx, int n, int L_max, int W, hipStream_t st);

// Automatic work split for side L: L itself (whole rows per wave) when L is
// a multiple of 32 and at most 1024, else a segment width (a multiple of 32,
// <= L - 32).
// Automatic segment widths: for launches over many lattices (ensembles,
// server) whole rows up to kEnsWholeRowMaxL; split_segw: rows cut into
// segments of about 1376 columns (a single lattice, which needs the waves).
constexpr int kEnsWholeRowMaxL = 8192;
int auto_segw(int L);
int split_segw(int L);
// Whether a width is usable at side L: a multiple of 32 up to L - 32
// (segments), or L itself when L is a multiple of 32 (whole rows).
bool segw_valid(int L, int segw);
// Fill in segw, nseg, rpw, stride, nw of a replica of side L (segw 0 =
// automatic; segw == L: whole rows, min(L / 4, max(1, 1024 / L)) per wave).
void ens_geometry(EnsRep& rp, int L, int segw);
// Waves of one launch for this replica, padded to whole workgroups of wpg waves.
int ens_waves(const EnsRep& rp, int wpg = kWavesPerGroup);
// LDS words one wave of this replica uses.
int ens_wave_words(const EnsRep& rp);
// Dynamic LDS of a workgroup of wpg waves of at most max_wave_words each.
size_t ens_lds_bytes(int max_wave_words, int wpg = kWavesPerGroup);
bool ens_wpg_valid(int wpg);
// Enqueue one chunk of `len` sweeps (len <= chunk) for the n replicas of
// d_reps on st: (if set_active) n_active = len for every replica, zero their
// counters, 4 segment launches per sweep (replicas run q < n_active), the
// per-replica scan into counts[n][chunk] (and rp.nc), the copy of the final
// state back to rp.lat when it lies in rp.lat2, the advance of t0.
hipError_t launch_ens_chunk(EnsRep* d_reps, int n, int total_waves, size_t lds, int len, int chunk,
                            bool set_active, unsigned long long* counts, hipStream_t st, int wpg = kWavesPerGroup,
                            unsigned long long* span = nullptr);
// The same chunk in three parts, for callers that bracket each segment
// launch (residue a of sweep q of the chunk) with events of their own.
hipError_t launch_ens_begin(EnsRep* d_reps, int n, int len, int chunk, bool set_active, hipStream_t st);
// span: NULL, or kSpanWords words: kSpanSlots (earliest start, latest end)
// pairs in wall-clock ticks, set to (~0, 0) beforehand, workgroup b updating
// pair b mod kSpanSlots -- a diagnostic of the launch's own span.  Spread so
// that the atomics of one address stay few.
constexpr int kSpanSlots = 256;
constexpr int kSpanWords = 2 * kSpanSlots;
hipError_t launch_ens_residue(const EnsRep* d_reps, int n, int total_waves, size_t lds, int a, int q,
                              hipStream_t st, int wpg = kWavesPerGroup, unsigned long long* span = nullptr);
hipError_t launch_ens_end(EnsRep* d_reps, int n, int chunk, unsigned long long* counts, hipStream_t st);
// One chunk of a tiled ensemble (pgg_tiled.hip): the same bookkeeping as
// launch_ens_chunk, 4 part launches per sweep over total_blocks workgroups
// (each replica's tiled_blocks(L), in replica order), in place.
hipError_t launch_ens_tiled_chunk(EnsRep* d_reps, int n, int total_blocks, int len, int chunk,
                                  unsigned long long* counts, hipStream_t st);
// Two residues per launch for one lattice (pgg_ensemble.hip, k_ens_pair):
// workgroups of kPairBand rows x one segment; d_rep holds the one replica.
constexpr int kPairBand = 32;
size_t pair_lds_bytes(int segw);
int pair_blocks(const EnsRep& rp);
// One chunk of len sweeps, 2 launches per sweep (residues 0-1, then 2-3).
hipError_t launch_pair_chunk(EnsRep* d_rep, int blocks, size_t lds, int len, int chunk, unsigned long long* counts,
                             hipStream_t st, unsigned long long* span);

// The automatic single-lattice plan of the segment paths (pgg_api.hip): for a
// bit-packed lattice of side L >= 64 with kernel AUTO and group 0, whether
// the paired kernel runs, and the segment width.
void auto_segment_plan(uint32_t L, int device, bool* pair, int* segw);

// Set n_launches span records (kSpanWords words each) to (~0, 0) pairs.
hipError_t launch_span_reset(unsigned long long* span, int n_launches, hipStream_t st);
// Set the sweep index t0 of every replica (graph-safe, no host memory).
hipError_t launch_ens_set_t0(EnsRep* d_reps, int n, uint32_t t0, hipStream_t st);

// Sets the calling thread's pgg_last_error() text (printf-style).
void set_errorf(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

}  // namespace pgg
