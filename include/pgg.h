/*
 * pgg.h -- C ABI of the MI355X (gfx950) spatial public goods game engine.
 *
 * The model is the spatial public goods game of M. Perc, "High-performance
 * parallel computing in the classroom using the public goods game as an
 * example" (2017), Sec. III: an L x L periodic square lattice of cooperators
 * (C = 1) and defectors (D = 0), overlapping von Neumann groups of G = 5,
 * cost c = 1, multiplication factor r (payoffs Eq. (1)-(2), summed over the
 * five groups a player belongs to), and imitation of a random nearest
 * neighbour with the Fermi probability of Eq. (3) at noise K.  The observable
 * is the cooperator fraction rho_C of Eq. (4).
 *
 * The engine advances the lattice with a deterministic sweep: one Monte
 * Carlo step (MCS) visits the 16 colour classes k = 4 (i mod 4) + (j mod 4),
 * k = 0..15 in order, and gives every site of class k one elementary step of
 * Sec. III.  Concurrently updated sites are at least 4 apart, beyond the
 * 3-line read radius of an elementary step (Sec. IV), so a colour class
 * updates in parallel without races.  Random numbers come from
 * Philox4x32-10 with key (seed mod 2^32, seed >> 32) and counter
 * (x, t, k, 0) for the elementary step of site x = i L + j in sweep t
 * (0-based), direction d = w0 >> 30 (0 E, 1 W, 2 S, 3 N), acceptance word
 * u = w1; the initial state uses counter (x, 0, 0, 1) and s_x = [w0 < P0],
 * P0 = min(2^32, floor(p0 2^32 + 1/2)).  A copy happens iff s_x != s_y and
 * u < T[dSigma + 25][ds + 1], T = min(2^32 - 1, floor(W 2^32 + 1/2)),
 * W = 1 / (1 + exp(((r dSigma)/5 - 5 ds)/K)) in binary64, where Sigma is the
 * sum of the cooperator counts of the five groups containing a player, so
 * that Pi = (r/5) Sigma - 5 s exactly.  Results are a pure function of
 * (parameters, t, lattice): identical for both storage layouts, every kernel
 * variant, chunking of sweeps into calls, batching and streams.
 *
 * Conventions for every call:
 *   - Every call returns pgg_status; 0 is success, negative is an error.
 *     No C++ exception crosses this boundary.  pgg_last_error() returns a
 *     thread-local description of the last error raised on the calling thread.
 *   - Arguments are validated before anything is allocated or launched; an
 *     invalid argument returns PGG_E_INVAL with no side effect.
 *   - A HIP error returns PGG_E_DEVICE and poisons the handle: every later
 *     call on it except pgg_destroy returns PGG_E_STATE.
 *   - A handle is not thread-safe; distinct handles may be used from distinct
 *     threads at once.  Work is ordered on the handle's HIP stream.  Graphs
 *     are captured in thread-local mode on a non-blocking stream (the
 *     handle's own, or the caller's); a caller stream given to an ensemble or
 *     server that captures graphs should be non-blocking, or another thread's
 *     work on the null stream may fail the capture.
 *   - "host" pointers are ordinary CPU memory owned by the caller; "device"
 *     pointers are HIP device memory on the current device.
 */
#ifndef PGG_H
#define PGG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PGG_OK = 0,
    PGG_E_INVAL = -1,  /* invalid argument; nothing was changed            */
    PGG_E_NOMEM = -2,  /* device or host allocation failed                 */
    PGG_E_DEVICE = -3, /* a HIP call failed; the handle is now poisoned    */
    PGG_E_STATE = -4   /* handle poisoned by an earlier device error       */
} pgg_status;

/* Storage of the strategy lattice in device memory.  Results are identical. */
typedef enum {
    PGG_LAYOUT_INT8 = 0, /* one byte per site (0 or 1), row-major, x = i L + j */
    PGG_LAYOUT_BITS = 1  /* one bit per site: column j of row i is bit (j mod
                            32) of 32-bit word j / 32 of the row; each row is
                            padded to a multiple of 64 bits with zero bits     */
} pgg_layout;

/* Sweep kernel selection (a tuning choice; results never depend on it). */
typedef enum {
    PGG_KERNEL_AUTO = 0,    /* SEGMENT_PAIR when its workgroups all fit the
                               device at once with one or two per CU (L = 4096
                               on 256 CUs) and group is 0; RESIDENT for L = 64,
                               96 and 128 with group 0; else SEGMENT for
                               L >= 64; below L = 64, COLOUR (int8) or
                               ROWBAND_COMPACT (bits)                            */
    PGG_KERNEL_COLOUR = 1,  /* int8 only: one launch per colour class, global
                               memory, every site evaluated (reference path)   */
    PGG_KERNEL_ROWBAND = 2, /* bits only: one launch per row residue i mod 4
                               (4 colour classes), rows staged in LDS, every
                               site evaluated                                    */
    PGG_KERNEL_ROWBAND_COMPACT = 3, /* bits only: as ROWBAND, but sites whose 4
                               neighbours all share their strategy are resolved
                               without drawing random numbers (their update is
                               a no-op), and the rest are packed densely onto
                               the lanes                                         */
    PGG_KERNEL_ROWBAND_STAGED = 4 /* bits only: as ROWBAND_COMPACT, but the random
                               numbers of all four colour classes of a launch are
                               drawn in one batch (for a superset of the sites
                               that can change) before the classes are updated;
                               needs 8 L R + O(L) bytes of LDS, so large L use
                               ROWBAND_COMPACT under AUTO; an explicit request
                               that does not fit is PGG_E_INVAL                 */,
    PGG_KERNEL_STRIP = 5    /* bits only: one persistent cooperative launch per
                               pgg_sweep call; each workgroup keeps a strip of
                               rows in LDS for all sweeps and exchanges 3-row
                               halos with its two neighbours through global
                               memory and progress flags (no grid barrier).
                               Waits are bounded: a neighbour that stops making
                               progress for ~4 s aborts the launch, and the call
                               that observes it returns PGG_E_DEVICE.  Needs the
                               same LDS footprint limit as ROWBAND_STAGED        */,
    PGG_KERNEL_SEGMENT = 6  /* L >= 64: one launch per row residue;
                               one wave per row segment, no workgroup barriers:
                               the wave copies the 7 rows it reads into a
                               private LDS window, runs the four colour classes
                               on the segment plus a margin of 9/6/3/0 columns
                               (recomputed by both neighbouring segments) and
                               writes back its own columns; sites without a
                               differing neighbour draw nothing.  With L a
                               multiple of 32 (automatic up to L = 1024, or
                               tile = L) a wave owns whole rows instead and
                               recomputes nothing.  int8 layout: the sweeps run
                               on a bit-packed working copy that the library
                               allocates (two bits-layout lattices); each
                               pgg_sweep call packs the int8 lattice into it
                               first and unpacks the result at its end        */,
    PGG_KERNEL_SEGMENT_PAIR = 7 /* L a multiple of 32, L >= 512: the
                               segment update with two row residues per launch
                               (two launches per sweep): a workgroup stages a
                               band of 32 rows plus 6 halo rows each side once,
                               runs residue a on its rows and the 3-row halos
                               (with 12 more margin columns), synchronises, and
                               runs residue a + 1 on its rows.  tile: segment
                               width, a multiple of 32 up to L - 64 (0 =
                               automatic); group must be 0.  int8 layout: as
                               for SEGMENT, through a bit-packed working copy */,
    PGG_KERNEL_RESIDENT = 8 /* L a multiple of 32, 64 <= L <= 512 (above
                               256 it takes more than 64 KB of LDS: the
                               device's per-workgroup limit decides): one
                               workgroup of `group` waves (4, 8 or 16; 0 =
                               automatic) keeps the whole lattice in
                               LDS (with 3 periodic halo rows above and below)
                               and runs every sweep of a pgg_sweep call chunk
                               (up to 4096 sweeps) in one launch: per row
                               residue the waves update its rows with the
                               whole-row update of SEGMENT, then a workgroup
                               barrier and a halo refresh.  One CU does the
                               work, so lattices on other streams can run
                               beside it.  tile must be 0.  int8
                               layout: through a bit-packed working copy, as
                               for the tiled schedule.  Timing mode times
                               one launch per chunk                             */
} pgg_kernel;

/* The update schedule: which dynamics a Monte Carlo step runs.  Unlike the
 * kernel, the schedule changes the results (different sites are updated in
 * a different order with different random numbers). */
typedef enum {
    PGG_SCHEDULE_COLOUR16 = 0, /* the 16-colour sublattice sweep: colours
                                  k = 4 (i mod 4) + (j mod 4) in ascending
                                  order, every site once per sweep; Philox
                                  counter (x, t, k, 0) per site            */
    PGG_SCHEDULE_TILED = 1     /* the double tiling of Sec. IV (Fig. 2): 4 x 4
                                  domains of four types, type 1 + 2 (I mod 2)
                                  + (J mod 2) for domain (I, J); a Monte Carlo
                                  step runs the types in turn, every domain of
                                  the running type taking 16 random sequential
                                  steps (x uniform in the domain, y uniform
                                  among its neighbours).  Step m of part p of
                                  domain (I, J) in sweep t uses the Philox
                                  counter (I L/4 + J, t, 16 p + m, 2): x =
                                  player w0 >> 28 of the domain (row-major),
                                  direction (w0 >> 26) mod 4, u = w1.  Needs
                                  L % 8 == 0, kernel AUTO, tile 0 and group
                                  0; on the int8 layout the steps run on a
                                  bit-packed working copy, as for SEGMENT  */
} pgg_schedule;

/* The game the players play.  Unlike the kernel, the game changes the
 * results. */
typedef enum {
    PGG_GAME_PUBLIC_GOODS = 0, /* the spatial public goods game of Sec. III
                                  (G = 5, c = 1, multiplication factor r)  */
    PGG_GAME_PAIRWISE_PD = 1   /* the pairwise prisoner's dilemma Sec. VI
                                  names as the next game for the scheme: each
                                  player plays its four nearest neighbours
                                  (the weak dilemma, our reading: R = 1 for C
                                  meeting C, T = b for D meeting C, S = P =
                                  0, with b = pgg_params.r) and imitates a
                                  random neighbour with the Fermi rule of
                                  Eq. (3).  An elementary step reads the
                                  radius-2 diamond around x, and a sweep runs
                                  8 colour classes -- the cosets of the
                                  sublattice spanned by (2, 2) and (4, 0):
                                  class k = 4 (i mod 2) + ((j - 2 h) mod 4),
                                  h = (i div 2) mod 2, k = 0..7 in order --
                                  with the Philox counter (x, t, k, 0), d =
                                  w0 >> 30, u = w1, and a copy iff s_x != s_y
                                  and u < T[(dir 5 + n_x) 5 + n_y] (dir 0: x
                                  is C, dir 1: x is D; n = cooperating
                                  neighbours; see pgg_pd_table).  Initial
                                  state as for the public goods game.  Needs
                                  schedule 0, kernel AUTO, tile 0, group 0;
                                  single handles only (not ensembles, the
                                  server or pgg_sweep_static)              */
} pgg_game;

/* Simulation parameters (Sec. III).  G = 5 and c = 1 are fixed. */
typedef struct {
    uint32_t L;      /* lattice side; 4 <= L <= 32768 and L % 4 == 0          */
    double r;        /* multiplication factor; finite, r >= 0 (paper: r > 1)  */
    double K;        /* Fermi noise of Eq. (3); finite, K > 0 (paper: 0.5)    */
    double p0;       /* initial cooperator fraction in [0, 1] (paper: 0.5)    */
    uint64_t seed;   /* Philox key                                            */
    uint32_t layout; /* pgg_layout                                            */
    uint32_t kernel; /* pgg_kernel; must match the layout unless AUTO         */
    uint32_t tile;   /* work split; 0 = chosen by the library.  STRIP: rows
                        per strip (>= 4); ROWBAND*: rows per band; SEGMENT:
                        columns per segment (a multiple of 32, <= L - 32),
                        or L itself: whole rows per wave (min(L/4, max(1,
                        1024/L)) of them when L is a multiple of 32, else one
                        periodic row).  A value
                        the kernel cannot use is PGG_E_INVAL.  Results never
                        depend on it.                                         */
    uint32_t group;  /* SEGMENT: segment waves per workgroup, 2, 4 or 8
                        (0 = 4); other kernels: must be 0.  Results never
                        depend on it.                                         */
    uint32_t schedule; /* pgg_schedule (0 = the 16-colour sweep)            */
    uint32_t game;     /* pgg_game (0 = the public goods game)              */
} pgg_params;

typedef struct pgg_sim pgg_sim; /* opaque handle */

/* Bytes of device memory the lattice of these parameters occupies (the size
 * a caller-supplied dev_buf must have).  0 if the parameters are invalid. */
size_t pgg_device_bytes(const pgg_params* p);

/* The plan pgg_init would take for p on the current device, without
 * allocating or launching: *kernel the pgg_kernel it runs (AUTO resolved;
 * PGG_KERNEL_AUTO for the tiled schedule and the pairwise game, which have a
 * kernel each) and *tile its work split -- segment width for SEGMENT and
 * SEGMENT_PAIR, rows per band for the ROWBAND kernels, waves per workgroup
 * for RESIDENT, the requested strip height for STRIP (0: chosen at
 * pgg_init from the device's occupancy), 0 for the others.  PGG_E_INVAL
 * for parameters pgg_init refuses on validation. */
pgg_status pgg_plan(const pgg_params* p, uint32_t* kernel, uint32_t* tile);

/* Create a simulation and draw its initial state (Sec. III: every player C
 * with probability p0, D otherwise), t = 0.
 *   p          host; copied, the caller keeps ownership.
 *   dev_buf    device buffer of >= pgg_device_bytes(p) bytes, 4-byte
 *              aligned, that will hold the lattice (e.g. a torch tensor's
 *              data_ptr()); it must stay valid until pgg_destroy.  NULL: the library allocates and
 *              owns the lattice memory.  Small per-handle buffers (the
 *              threshold table, counters, count history) are always
 *              allocated by the library.
 *   dev_bytes  size of dev_buf (ignored when dev_buf is NULL).
 *   hip_stream hipStream_t to order all work on; NULL = the null stream.
 *   out        host; receives the handle (set to NULL on error).
 * Synchronises the stream once (to read N_C(0)). */
pgg_status pgg_init(const pgg_params* p, void* dev_buf, size_t dev_bytes, void* hip_stream,
                    pgg_sim** out);

/* Advance n_sweeps Monte Carlo steps (one sweep = the 16 colour classes)
 * from the current sweep index t; afterwards t += n_sweeps.  Requires
 * t + n_sweeps <= 2^32.
 *   coop_counts  host array of n_sweeps entries receiving N_C(t+1) ... N_C(t+n)
 *                (the Eq. (4) sum after each sweep), or NULL.
 * With coop_counts == NULL the call only enqueues work on the stream and
 * returns; with it, the call synchronises the stream. n_sweeps == 0 is a
 * no-op. */
pgg_status pgg_sweep(pgg_sim* s, uint32_t n_sweeps, uint64_t* coop_counts);

/* rho = N_C(t) / L^2 after the last completed sweep (Eq. (4) without the
 * time average).  Synchronises the stream. rho: host. */
pgg_status pgg_density(pgg_sim* s, double* rho);

/* N_C(t), the number of cooperators.  Synchronises the stream. n_c: host. */
pgg_status pgg_coop_count(pgg_sim* s, uint64_t* n_c);

/* The current sweep index t (number of sweeps completed).  Host only. */
pgg_status pgg_sweep_index(const pgg_sim* s, uint64_t* t);

/* Copy the lattice to host_LxL (host, L*L bytes, row-major, values 0/1).
 * Synchronises the stream. */
pgg_status pgg_read_lattice(pgg_sim* s, uint8_t* host_LxL);

/* Replace the lattice by host_LxL (host, L*L bytes of 0/1; any other byte
 * value is PGG_E_INVAL) and set the sweep index to t (t <= 2^32), e.g. to
 * resume from a checkpoint.  Synchronises the stream. */
pgg_status pgg_write_lattice(pgg_sim* s, const uint8_t* host_LxL, uint64_t t);

/* Copy the 153 Fermi thresholds T[(dSigma + 25) * 3 + ds + 1] that the
 * device uses to host_T (host, 153 entries; for the pairwise game the 50 of
 * pgg_pd_table, then zeros).  Synchronises the stream. */
pgg_status pgg_threshold_table(pgg_sim* s, uint32_t* host_T);

/* The Fermi thresholds of Eq. (3) for (r, K), as every handle, ensemble
 * replica and served job of the library uses them: T[(dSigma + 25) * 3 +
 * ds + 1] = min(2^32 - 1, floor(W 2^32 + 1/2)) with W = 1 / (1 + exp(((r
 * dSigma)/5 - 5 ds)/K)), dSigma in [-25, 25], ds in {-1, 0, 1}, evaluated
 * on the host in binary64 in exactly this operation order with the C
 * library's exp (Sec. III; with c = 1 and G = 5, Pi_x - Pi_y = (r/5) dSigma
 * - 5 ds).  host_T: host, 153 entries.  r finite and >= 0, K finite and >
 * 0, else PGG_E_INVAL.  Host only: no device, no handle. */
pgg_status pgg_fermi_table(double r, double K, uint32_t* host_T);

/* The 50 thresholds of the pairwise prisoner's dilemma (PGG_GAME_PAIRWISE_PD)
 * for temptation b and noise K, as the library uses them: T[(dir * 5 + n_x)
 * * 5 + n_y] = min(2^32 - 1, floor(W 2^32 + 1/2)), W = 1 / (1 + exp((Pi_x -
 * Pi_y) / K)), with Pi_x = n_x and Pi_y = b n_y for dir 0 (x cooperates, y
 * defects) and Pi_x = b n_x, Pi_y = n_y for dir 1 (x defects, y
 * cooperates); n_x, n_y in 0..4 count the cooperating neighbours; binary64
 * on the host in this operation order with the C library's exp.  host_T:
 * host, 50 entries.  b finite and >= 0, K finite and > 0, else
 * PGG_E_INVAL.  Host only.  pgg_threshold_table of a pairwise-game handle
 * returns these 50 entries followed by zeros. */
pgg_status pgg_pd_table(double b, double K, uint32_t* host_T);

/* Diagnostics for measurement.  With enable != 0, later pgg_sweep calls on
 * this handle time their sweep-kernel launches with HIP events on the
 * handle's stream and count the site updates that drew random numbers.
 * Row-band, strip and colour kernels: a pair of events around every launch.
 * Segment kernel: its graph replays (timing mode has graphs of its own)
 * are bracketed per chunk, the stream is synchronised after every chunk,
 * and every launch records its own span (see pgg_kernel_span).  Resets the
 * totals.  Timing adds work, so a throughput measurement should run with it
 * disabled.  Synchronises the stream. */
pgg_status pgg_set_kernel_timing(pgg_sim* s, int enable);

/* Totals since the last pgg_set_kernel_timing: number of timed sweep-kernel
 * launches, their summed event-to-event duration in ms (segment kernel: of
 * the chunks holding them, with the chunks' bookkeeping kernels), and the
 * number of site updates that drew random numbers (0 for the colour kernel
 * and the tiled schedule, where every update draws, and for the pairwise
 * game, which does not count them).
 * All three pointers are host and must be non-NULL.  Synchronises. */
pgg_status pgg_kernel_timing(pgg_sim* s, uint64_t* launches, double* total_ms, uint64_t* drawn);

/* Segment kernel, totals since the last pgg_set_kernel_timing: number of
 * timed launches and the sum over them of the launch's own span -- latest
 * workgroup end minus earliest workgroup start, read from the device wall
 * clock.  0 launches for the other kernels.  Host pointers, non-NULL.
 * Host only. */
pgg_status pgg_kernel_span(pgg_sim* s, uint64_t* launches, double* total_us);

/* Diagnostics for failure handling: the longest time (seconds, >= 0) a
 * workgroup of the STRIP kernel waits for a neighbouring strip before it
 * aborts the launch (default 4).  0 makes almost every wait abort, which
 * lets a test exercise the abort path: the launch then ends early on every
 * workgroup, and the next synchronising call returns PGG_E_DEVICE and
 * poisons the handle.  Other kernels ignore it.  Host only. */
pgg_status pgg_set_strip_wait(pgg_sim* s, double seconds);

/* Release the handle and every buffer the library allocated.  Never frees a
 * caller-supplied dev_buf.  NULL is a no-op.  Synchronises the stream. */
void pgg_destroy(pgg_sim* s);

/* ------------------------------------------------------------------------
 * Batched ensembles: many independent lattices (replicas) of uneven L, r
 * and seed -- the ensembles the absorbing-phase-transition analysis of
 * Sec. V averages over -- advanced together.  Every launch covers one row
 * residue of one sweep of every replica (the segment kernel's work split,
 * replica by replica), and a chunk of sweeps is captured once in a hipGraph
 * and replayed.  Each replica's lattice and counts are exactly those of a
 * pgg_init / pgg_sweep run with the same parameters.
 * ------------------------------------------------------------------------ */
typedef struct pgg_ensemble pgg_ensemble; /* opaque; not thread-safe */

/* Tuning of a batched launch: what only changes the speed, never a result.
 *   tiles      NULL (automatic) or host array of n_reps work splits as
 *              pgg_params.tile of the segment kernel (0 = automatic: whole
 *              rows up to L = 8192, segments of about 1376 columns above;
 *              a single lattice's automatic split keeps segments above
 *              L = 1024 and for L not a multiple of 32, where it needs the
 *              waves).
 *   chunk      sweeps per graph replay, 1..1024 (device counters hold
 *              chunk x n_reps x 4 KiB).
 *   waves_per_group  segment waves per workgroup: 2, 4 or 8 (0 = 4).  A
 *              workgroup serves one replica and shares one copy of its
 *              threshold table; each replica's waves are padded to whole
 *              workgroups.
 *   branches   concurrent replica groups, 0..16 (0: two for the 16-colour
 *              schedule, one for the tiled one; 1: one): the replicas
 *              swept by segments are cut into this many contiguous ranges
 *              of about equal work (sum of L^2), each range's chunk is its
 *              own chain of launches, and the chains run side by side as
 *              parallel branches of the chunk's graph.  The tiled schedule
 *              takes 0 or 1.
 *   resident_max_L  0, or a side in [64, 512]: replicas with L a multiple of
 *              32 up to this side are swept by the resident kernel instead
 *              -- one workgroup per replica holds its lattice in LDS and
 *              runs the whole chunk in one launch -- as one more parallel
 *              branch beside the segment launches (16-colour schedule).
 *   resident_waves  waves per resident workgroup: 4, 8 or 16 (0 = 8). */
typedef struct {
    const uint32_t* tiles;
    uint32_t chunk;
    uint32_t waves_per_group;
    uint32_t branches;
    uint32_t resident_max_L;
    uint32_t resident_waves;
} pgg_ensemble_tune;

/* Create n_reps replicas and draw their initial states (t = 0).
 *   reps       host array of n_reps parameter sets: 64 <= L <= 32768, L % 4
 *              == 0, layout BITS, kernel AUTO or SEGMENT, group 0, game 0,
 *              and one schedule for all of them; copied.  With
 *              PGG_SCHEDULE_TILED (L % 8 == 0) every launch covers one
 *              domain type of one step of every replica, in place, and only
 *              tune->chunk applies (tiles NULL or all 0).
 *   tune       host, NULL for the defaults (chunk 32, everything else
 *              automatic), else the tuning above; copied.
 *   hip_stream stream to order the work on; NULL: the ensemble creates and
 *              owns a stream of default priority (graphs cannot capture the
 *              null stream).
 * Synchronises the stream once. */
pgg_status pgg_ensemble_create(const pgg_params* reps, uint32_t n_reps, const pgg_ensemble_tune* tune,
                               void* hip_stream, pgg_ensemble** out);

/* Advance every replica n_sweeps sweeps.  counts: NULL, or host array of
 * n_reps rows of n_sweeps entries receiving N_C after each sweep (row k is
 * replica k).  Synchronises once per chunk when counts != NULL. */
pgg_status pgg_ensemble_sweep(pgg_ensemble* e, uint32_t n_sweeps, uint64_t* counts);

/* N_C(t) of every replica into host n_c[n_reps].  Synchronises. */
pgg_status pgg_ensemble_coop_counts(pgg_ensemble* e, uint64_t* n_c);

/* The common sweep index t of the replicas.  Host only. */
pgg_status pgg_ensemble_sweep_index(const pgg_ensemble* e, uint64_t* t);

/* Lattice of replica rep into host_LxL (L*L bytes, row-major 0/1).
 * Synchronises. */
pgg_status pgg_ensemble_read_lattice(pgg_ensemble* e, uint32_t rep, uint8_t* host_LxL);

/* The 153 Fermi thresholds replica rep uses on the device (the layout of
 * pgg_fermi_table) into host_T.  Synchronises. */
pgg_status pgg_ensemble_threshold_table(pgg_ensemble* e, uint32_t rep, uint32_t* host_T);

/* Release every buffer, graph and owned stream.  NULL is a no-op. */
void pgg_ensemble_destroy(pgg_ensemble* e);

/* Autotune the batched launch for a set of replicas: the segment width of
 * each distinct L, the waves per workgroup, the concurrent replica groups,
 * the resident sweep of small replicas and the chunk length of a graph
 * replay.  Results never depend on them; only the speed does.
 *   reps, n_reps  as for pgg_ensemble_create, schedule COLOUR16 (the tiled
 *                 schedule has nothing to tune: PGG_E_INVAL).
 *   probe_sweeps  sweeps per timed run, 1..4096; at least 64 and twice the
 *                 trial's chunk are run.
 *   hip_stream    as for pgg_ensemble_create.
 *   tiles_out     host array of n_reps: the chosen width of each replica
 *                 (equal for equal L).
 *   tune_out      host: the chosen tuning (its tiles point at tiles_out).
 *   ms_out        NULL, or the best time per sweep of the whole ensemble.
 * Trials run on trial ensembles created from reps (fresh initial states
 * each): first the width of each distinct L in turn (the six with the
 * most work, sum of L^2, in that order; others automatic) over the doublings
 * 64, 128, ... below L - 32, L - 32 rounded down to a multiple of 32, and
 * whole rows (L), the other sizes held at their
 * best so far, then the waves per workgroup over 2, 4, 8, then the
 * concurrent groups over 1, 2, 4 together with resident sweeps off, up to
 * L = 128 or 256 (when some replica fits), then their 4, 8 or 16
 * waves, then the chunk over 8, 16, 32, 64, 128; each trial runs once
 * untimed and keeps its best of three timed runs.  Every trial's final
 * cooperator counts must equal those of the first trial of the same length, else
 * PGG_E_DEVICE with a message (a tuning-dependent result would be a bug).
 * Needs the device memory of one trial ensemble at chunk 128. */
pgg_status pgg_ensemble_autotune(const pgg_params* reps, uint32_t n_reps, uint32_t probe_sweeps,
                                 void* hip_stream, uint32_t* tiles_out, pgg_ensemble_tune* tune_out,
                                 double* ms_out);



/* One batched run from the initial states: create the ensemble of reps,
 * advance every replica n_sweeps sweeps, release it.  counts: NULL, or host
 * array of n_reps rows of n_sweeps entries (N_C after each sweep, row k =
 * replica k).  tune: NULL to autotune first (pgg_ensemble_autotune with 8
 * probe sweeps; the tiled schedule takes the defaults), else the settings
 * to use.  Each replica's counts are those of pgg_init + pgg_sweep with its
 * parameters.  Synchronises. */
pgg_status pgg_ensemble_run(const pgg_params* reps, uint32_t n_reps, uint32_t n_sweeps, uint64_t* counts,
                            const pgg_ensemble_tune* tune, void* hip_stream);

/* ------------------------------------------------------------------------
 * Job server: continuous batching of simulation jobs on one GPU.  Jobs are
 * submitted at any time and queue on the host.  Each pgg_server_step
 * (1) admits queued jobs in arrival order while their device footprint
 * (pgg_server_job_bytes) fits the HBM budget, then any later job that still
 * fits (backfill), drawing their initial states on the device; (2) advances
 * every resident job by min(chunk, remaining) sweeps in the same launches,
 * each at its own sweep index, replayed from a hipGraph captured once per
 * bucket of resident-replica slots and waves (idle replicas pad the table);
 * (3) copies the chunk's counts out and retires finished jobs (final
 * lattices copied out with one synchronisation, device space freed).  Lattices
 * stay resident for a job's whole life.  A job's counts and final lattice
 * are exactly those of pgg_init + pgg_sweep with the same parameters.
 * Not thread-safe; one server per thread.
 * ------------------------------------------------------------------------ */
typedef struct pgg_server pgg_server;

typedef struct {
    uint32_t queued;       /* jobs waiting for admission                    */
    uint32_t resident;     /* jobs on the device                            */
    uint64_t completed;    /* jobs finished since creation                  */
    uint64_t bytes_in_use; /* device bytes held by resident jobs            */
    uint64_t peak_bytes;   /* largest bytes_in_use so far (<= budget)       */
    uint64_t budget;       /* the HBM budget (rounded down to 256 B)        */
    uint64_t site_updates; /* L^2 x sweeps completed, over all jobs         */
} pgg_server_info;

/* Device bytes a job of side L occupies under a server with this chunk:
 * lattice (bit-packed), threshold table, per-sweep counters, N_C. */
size_t pgg_server_job_bytes(uint32_t L, uint32_t chunk);

/* Create a server.
 *   hbm_budget    device bytes for resident jobs (one arena, allocated now);
 *                 must hold at least the footprint of an L = 64 job.
 *   max_L         largest L accepted (multiple of 4 in [64, 32768]); sizes a
 *                 max_L^2-byte read-out buffer allocated outside the budget.
 *   max_resident  most jobs on the device at once (1..65536).
 *   chunk         sweeps per step (1..1024).
 *   hip_stream    stream to order work on; NULL: the server owns one.
 * Fails with PGG_E_NOMEM if the device cannot hold the arena. */
pgg_status pgg_server_create(size_t hbm_budget, uint32_t max_L, uint32_t max_resident, uint32_t chunk,
                             void* hip_stream, pgg_server** out);

/* Queue a job: p (host, copied; 64 <= L <= max_L, layout BITS, kernel AUTO
 * or SEGMENT, schedule COLOUR16, game 0; tile 0 or a segment width whose
 * LDS fits the server's launches, which reserve the widest automatic layout
 * up to max_L) and n_sweeps >= 1.  A job whose footprint exceeds the whole
 * budget is PGG_E_INVAL.  job_id (host) receives its id.  Host only. */
pgg_status pgg_server_submit(pgg_server* s, const pgg_params* p, uint32_t n_sweeps, uint64_t* job_id);

/* One step (admit, run one chunk, retire).  n_resident (host, or NULL)
 * receives the number of jobs that ran in this step.  Synchronises. */
pgg_status pgg_server_step(pgg_server* s, uint32_t* n_resident);

/* Ids of jobs that finished since the last call (at most cap, oldest
 * first) into host ids; n receives how many.  Host only. */
pgg_status pgg_server_completed(pgg_server* s, uint64_t* ids, uint32_t cap, uint32_t* n);

/* State of a job: 0 queued, 1 on the device, 2 finished; sweeps done. */
pgg_status pgg_server_job_state(pgg_server* s, uint64_t id, int* state, uint32_t* sweeps_done);

/* Results of a finished job: counts (host, n_sweeps entries: N_C after each
 * sweep) and lattice (host, L*L bytes 0/1), each may be NULL.  Releases the
 * job's record: a second call is PGG_E_INVAL. */
pgg_status pgg_server_job_result(pgg_server* s, uint64_t id, uint64_t* counts, uint8_t* lattice);

pgg_status pgg_server_stats(const pgg_server* s, pgg_server_info* st);

/* Release the arena, the buffers and an owned stream.  NULL is a no-op. */
void pgg_server_destroy(pgg_server* s);

/* ------------------------------------------------------------------------
 * A sweep that allocates nothing, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It advances a caller's bit-packed lattice exactly as
 * pgg_init + pgg_sweep would (the same kernels, chosen as AUTO does), with
 * every buffer the kernels need beyond the caller's lattice and counts --
 * the Fermi thresholds, the per-sweep counters, the second lattice buffer
 * of the out-of-place sweep -- in one fixed device array of the library
 * (pgg_sweep_static_scratch_bytes() bytes, about 2.3 MB, held on each device
 * the call runs on until the process ends).  It calls no hipMalloc, hipFree
 * or allocating library routine, and does not synchronise.
 * ------------------------------------------------------------------------ */

/* Bytes of the fixed device array pgg_sweep_static uses on each device. */
size_t pgg_sweep_static_scratch_bytes(void);

/* Advance the lattice in dev_lattice n_sweeps sweeps from sweep index t0.
 *   p            host; L a multiple of 4 in [64, 4096] (larger L would need
 *                more than the fixed array: PGG_E_INVAL), r, K and seed as
 *                for pgg_init (p0 unused), layout BITS, kernel AUTO, tile 0,
 *                group 0, schedule COLOUR16; anything else is PGG_E_INVAL.
 *   dev_lattice  device, pgg_device_bytes(p) bytes, 4-byte aligned: the
 *                lattice in the bits layout (padding bits zero), updated in
 *                place; it holds the state after t0 sweeps on entry.
 *   t0           sweep index of that state; t0 + n_sweeps <= 2^32.
 *   dev_counts   device array of n_sweeps entries (8-byte aligned)
 *                receiving N_C after each sweep, or NULL.
 *   hip_stream   stream to order the work on (NULL: the null stream).
 * Only enqueues work.  Every call on a device shares that device's array,
 * which keeps the last call's contents (each call re-initialises what it
 * reads): calls that overlap on one device -- on different streams, or from
 * different threads -- race and give wrong results; order them on one
 * stream.  A launch error returns PGG_E_DEVICE (there is no handle to
 * poison). */
pgg_status pgg_sweep_static(const pgg_params* p, void* dev_lattice, uint64_t t0, uint32_t n_sweeps,
                            uint64_t* dev_counts, void* hip_stream);

/* Thread-local, NUL-terminated description of the last error on this thread
 * ("" if none).  Valid until the next call on this thread. */
const char* pgg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PGG_H */
