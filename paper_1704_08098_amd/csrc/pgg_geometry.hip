// Host-side geometry of the segment kernels: the automatic work split per
// side L (whole rows or segments), the per-replica wave counts and LDS
// footprints the launchers and the engines size their launches with.  Kept
// apart from the kernels so that a change of policy here leaves the kernel
// sources (and the profiles taken on them) as they are.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pgg_fullrow.hpp"
#include "pgg_internal.hpp"
#include "pgg_segment.hpp"

namespace pgg {

int split_segw(int L) {
    // About 1376 columns: at the drawn fraction of a lattice near r_c (about
    // 15 % of the sites) a class then lists about 50 sites, most of one
    // 64-lane pass; the row is split into equal segments of that order.  A
    // segment is at most L - 32 columns, so a row always takes two or more:
    // split it evenly (one segment of L - 32 columns and one of the rest
    // would leave the second wave almost empty).
    const int nseg = std::max(2, (L + 1375) / 1376);
    int w = (L / nseg + 31) & ~31;
    const int cap = (L - 32) & ~31;
    if (w > cap) w = cap;
    if (w < 32) w = 32;
    return w;
}

int auto_segw(int L) {
    // Whole rows: several per wave for L a multiple of 32 below 1024, else
    // one row per wave (periodic when L is not a multiple of 32).  A launch
    // over many lattices has waves to spare, so fewer, fuller waves win: a
    // row split into segments lists fewer sites per class for the same
    // per-class cost and recomputes its margins (ensembles of 64 replicas:
    // 2.0-2.6e11 -> 3.7-3.8e11 site updates/s at L = 500 ... 1020, 3.3-3.6e11
    // -> 4.9-5.4e11 at L = 1276 ... 1500, 1.6 x at 9 x L = 4096).  Up to L =
    // 8192 (62 KB of LDS for 4 waves per workgroup).
    if (L <= kEnsWholeRowMaxL) return L;
    return split_segw(L);
}

bool segw_valid(int L, int segw) {
    if (segw == L) return true;  // whole rows
    return segw > 0 && segw % 32 == 0 && segw + 32 <= L;
}

void ens_geometry(EnsRep& rp, int L, int segw) {
    if (segw == 0) segw = auto_segw(L);
    rp.L = L;
    rp.stride = 2 * ((L + 63) / 64);
    rp.nw = (L + 31) / 32;
    rp.segw = segw;
    if (segw == L && L % 32 == 0) {
        rp.nseg = 1;
        const int R = L >= 1024 ? 1 : 1024 / L;
        rp.rpw = R < L / 4 ? R : L / 4;
    } else {  // segments, or one periodic row per wave (segw == L)
        rp.nseg = (L + segw - 1) / segw;
        rp.rpw = 0;
    }
}

int ens_waves(const EnsRep& rp, int wpg) {
    if (rp.resident) return 0;  // swept by the resident kernel
    const int rows = rp.L / 4;
    const int wv = rp.rpw > 0 ? (rows + rp.rpw - 1) / rp.rpw : rows * rp.nseg;
    return (wv + wpg - 1) / wpg * wpg;
}

int ens_wave_words(const EnsRep& rp) { return rep_wave_words(rp); }

size_t ens_lds_bytes(int max_wave_words, int wpg) {
    return (kSegTableWords + (size_t)wpg * max_wave_words) * sizeof(uint32_t);
}

bool ens_wpg_valid(int wpg) { return wpg == 2 || wpg == 4 || wpg == 8; }

size_t pair_lds_bytes(int segw) {
    return (kSegTableWords + (size_t)(kPairBand + 12) * seg_window_words(segw) +
            (size_t)(kPairBand / 4 + 1) * seg_list_cap(segw)) * sizeof(uint32_t);
}

int pair_blocks(const EnsRep& rp) { return (rp.L + kPairBand - 1) / kPairBand * rp.nseg; }

}  // namespace pgg
