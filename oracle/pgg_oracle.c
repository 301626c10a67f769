/*
 * Oracle for the spatial public goods game (PGG) strategy-update sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source with the HIP library.
 *
 * Plain, single-threaded, deliberately slow C99.  Every function below states
 * the passage of the paper (M. Perc, "High-performance parallel computing in
 * the classroom using the public goods game as an example", 2017) it follows.
 *
 * Model (Sec. III): L x L periodic square lattice, strategies s in {D=0, C=1},
 * overlapping von Neumann groups of G = 5, cost c = 1, multiplication factor
 * r; group payoffs Eq. (1) (cooperator) and Eq. (2) (defector); the payoff of
 * a player is summed over the five groups it belongs to; the player imitates a
 * random nearest neighbour with the Fermi probability of Eq. (3).
 *
 * Three oracles:
 *   A  pgg_ref_sweep   the deterministic 16-colour sublattice sweep with a
 *                      Philox4x32-10 counter RNG and an integer acceptance
 *                      table.  This is the bit-exact contract.
 *   B  pgg_ref_rs_run  the textbook random-sequential Monte Carlo step of
 *                      Sec. III, payoffs from Eq. (1)-(2) group by group in
 *                      binary64, Eq. (3) in binary64.  Statistical check only.
 *   C  pgg_ref_sweep_tiled  the paper's own parallel dynamics, the double
 *                      tiling of Sec. IV (4 x 4 domains of four types, random
 *                      sequential steps inside each domain), with the same
 *                      counter RNG and table as A.  The bit-exact contract of
 *                      the tiled schedule.
 *   D  pgg_ref_pd_sweep  the pairwise prisoner's dilemma Sec. VI names as the
 *                      next game for the scheme: four pairwise games per
 *                      player, the same imitation, an 8-colour schedule.
 *
 * Conventions the paper leaves open (our reading, fixed here):
 *   - lattice index x = i*L + j, i = row, j = column, both periodic mod L;
 *   - colour of (i, j) is k = 4*(i mod 4) + (j mod 4); a sweep runs the
 *     colours k = 0..15 in ascending order; L must be a multiple of 4;
 *   - Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with key
 *     (seed mod 2^32, seed >> 32); update counter (x, t, k, 0) where t is the
 *     0-based index of the sweep; initial-state counter (x, 0, 0, 1);
 *   - neighbour direction d = w0 >> 30 selects y = (i, j+1), (i, j-1),
 *     (i+1, j), (i-1, j) for d = 0, 1, 2, 3; the acceptance word is u = w1;
 *   - a copy happens iff s_x != s_y and u < T[dSigma + 25][ds + 1] where
 *     T = min(2^32 - 1, floor(W * 2^32 + 1/2)) and W is Eq. (3) in binary64;
 *   - initial strategy s_x = [w0 < P0], P0 = min(2^32, floor(p0 * 2^32 + 1/2)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PGG_REF_OK 0
#define PGG_REF_EINVAL (-1)
#define PGG_REF_ENOMEM (-2)

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2,  */
/* 3", SC'11).  A round multiplies counter words 0 and 2 by two fixed odd    */
/* 32-bit constants, keeps both halves of the 64-bit products, and mixes the */
/* high halves with the other two counter words and the round key; the key  */
/* is advanced by two fixed Weyl increments between rounds.                  */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_MUL_A = 0xD2511F53u; /* multiplies word 0 */
static const uint32_t PHILOX_MUL_B = 0xCD9E8D57u; /* multiplies word 2 */
static const uint32_t PHILOX_WEYL_0 = 0x9E3779B9u; /* golden ratio */
static const uint32_t PHILOX_WEYL_1 = 0xBB67AE85u; /* sqrt(3) - 1 */

void pgg_ref_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL_0;
            k1 += PHILOX_WEYL_1;
        }
        uint64_t pa = (uint64_t)PHILOX_MUL_A * (uint64_t)c0;
        uint64_t pb = (uint64_t)PHILOX_MUL_B * (uint64_t)c2;
        uint32_t pa_hi = (uint32_t)(pa >> 32), pa_lo = (uint32_t)pa;
        uint32_t pb_hi = (uint32_t)(pb >> 32), pb_lo = (uint32_t)pb;
        uint32_t n0 = pb_hi ^ c1 ^ k0;
        uint32_t n1 = pb_lo;
        uint32_t n2 = pa_hi ^ c3 ^ k1;
        uint32_t n3 = pa_lo;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_site(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                        uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    pgg_ref_philox(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Lattice helpers                                                          */
/* ------------------------------------------------------------------------ */
static int wrap(int64_t a, int L)
{
    int64_t m = a % L;
    return (int)(m < 0 ? m + L : m);
}

static uint8_t at(const uint8_t* s, int L, int64_t i, int64_t j)
{
    return s[(size_t)wrap(i, L) * (size_t)L + (size_t)wrap(j, L)];
}

/* The von Neumann neighbourhood N[c]: the site itself and its four nearest
 * neighbours (Sec. III, Fig. 1 groups of G = 5). */
static const int NB_DI[5] = {0, 0, 0, 1, -1};
static const int NB_DJ[5] = {0, 1, -1, 0, 0};

/* Number of cooperators N_C in the group centred on (ci, cj) (Sec. III). */
int pgg_ref_group_nc(const uint8_t* s, int L, int ci, int cj)
{
    int n = 0;
    for (int m = 0; m < 5; ++m) n += at(s, L, (int64_t)ci + NB_DI[m], (int64_t)cj + NB_DJ[m]);
    return n;
}

/* Payoff of the player at (i, j) literally from Eq. (1)-(2): for each of the
 * G = 5 groups the player belongs to (centred on itself and on each of its
 * four neighbours, Fig. 1), add r*c*N_C/G, minus c if the player cooperates;
 * the total is the sum over the groups.  binary64, c = 1, G = 5. */
double pgg_ref_payoff(const uint8_t* s, int L, double r, int i, int j)
{
    const double G = 5.0, c = 1.0;
    const int coop = at(s, L, i, j);
    double total = 0.0;
    for (int g = 0; g < 5; ++g) {
        int nc = pgg_ref_group_nc(s, L, i + NB_DI[g], j + NB_DJ[g]);
        double pi_g = r * c * (double)nc / G; /* Eq. (2), defector share */
        if (coop) pi_g -= c;                   /* Eq. (1), cooperator pays c */
        total += pi_g;
    }
    return total;
}

/* Sigma_x = sum over the five groups containing x of their cooperator
 * counts.  With c = 1 and G = 5, Eq. (1)-(2) summed over the groups give
 * Pi_x = (r/5) * Sigma_x - 5 * s_x, an exact integer re-statement used by the
 * acceptance table.  Sites are indexed modulo L on every access, so at tiny L
 * a site reached twice is counted twice. */
int pgg_ref_sigma(const uint8_t* s, int L, int i, int j)
{
    int sigma = 0;
    for (int g = 0; g < 5; ++g) sigma += pgg_ref_group_nc(s, L, i + NB_DI[g], j + NB_DJ[g]);
    return sigma;
}

/* ------------------------------------------------------------------------ */
/* Fermi acceptance table, Eq. (3)                                          */
/* ------------------------------------------------------------------------ */
/* T[(dSigma + 25) * 3 + (ds + 1)] for dSigma = Sigma_x - Sigma_y in [-25, 25]
 * and ds = s_x - s_y in {-1, 0, 1}.  Pi_x - Pi_y = (r/5) dSigma - 5 ds, and
 * Eq. (3) gives W = 1 / (1 + exp((Pi_x - Pi_y) / K)).  The table holds
 * min(2^32 - 1, floor(W * 2^32 + 1/2)); a uniform 32-bit word u accepts iff
 * u < T.  Operation order in binary64 is part of the contract. */
int pgg_ref_table(double r, double K, uint32_t* T)
{
    if (!(isfinite(r) && r >= 0.0 && isfinite(K) && K > 0.0)) return PGG_REF_EINVAL;
    for (int dsig = -25; dsig <= 25; ++dsig) {
        for (int ds = -1; ds <= 1; ++ds) {
            double dpi = (r * (double)dsig) / 5.0 - 5.0 * (double)ds;
            double w = 1.0 / (1.0 + exp(dpi / K));
            double scaled = floor(w * 4294967296.0 + 0.5);
            uint32_t v = scaled >= 4294967295.0 ? 4294967295u : (uint32_t)scaled;
            T[(dsig + 25) * 3 + (ds + 1)] = v;
        }
    }
    return PGG_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Validation                                                               */
/* ------------------------------------------------------------------------ */
static int valid_L(uint32_t L) { return L >= 4 && L <= 32768 && (L % 4) == 0; }

/* ------------------------------------------------------------------------ */
/* Initial state (Sec. III: each player C or D with equal probability;      */
/* generalised to a cooperator fraction p0).                                */
/* ------------------------------------------------------------------------ */
int pgg_ref_init(uint32_t L, double p0, uint64_t seed, uint8_t* s, uint64_t* nc_out)
{
    if (!valid_L(L) || !(p0 >= 0.0 && p0 <= 1.0)) return PGG_REF_EINVAL;
    double pscaled = floor(p0 * 4294967296.0 + 0.5);
    uint64_t P0 = pscaled >= 4294967296.0 ? 4294967296ull : (uint64_t)pscaled;
    uint64_t nc = 0;
    for (uint32_t i = 0; i < L; ++i) {
        for (uint32_t j = 0; j < L; ++j) {
            uint32_t x = i * L + j, w[4];
            philox_site(seed, x, 0u, 0u, 1u, w);
            uint8_t v = (uint64_t)w[0] < P0 ? 1 : 0;
            s[(size_t)x] = v;
            nc += v;
        }
    }
    if (nc_out) *nc_out = nc;
    return PGG_REF_OK;
}

uint64_t pgg_ref_count(const uint8_t* s, uint32_t L)
{
    uint64_t n = 0;
    for (size_t x = 0; x < (size_t)L * L; ++x) n += s[x];
    return n;
}

/* ------------------------------------------------------------------------ */
/* Oracle A: one elementary step (Sec. III) at site (i, j) of colour k in    */
/* sweep t, then the 16-colour sweep.                                        */
/* ------------------------------------------------------------------------ */
static const int DIR_DI[4] = {0, 0, 1, -1}; /* d = 0: E, 1: W, 2: S, 3: N */
static const int DIR_DJ[4] = {1, -1, 0, 0};

/* The imitation of Sec. III for player x = (i, j), its neighbour in
 * direction d and the uniform 32-bit word u.  Returns +1 if x turned C, -1 if
 * it turned D, 0 if unchanged. */
static int imitate(uint8_t* s, int L, const uint32_t* T, int i, int j, int d, uint32_t u)
{
    const int yi = wrap((int64_t)i + DIR_DI[d], L), yj = wrap((int64_t)j + DIR_DJ[d], L);
    /* x plays in its five groups and earns Pi_x; y likewise (Eq. (1)-(2)). */
    const int sig_x = pgg_ref_sigma(s, L, i, j);
    const int sig_y = pgg_ref_sigma(s, L, yi, yj);
    const int sx = s[(size_t)i * L + j], sy = s[(size_t)yi * L + yj];
    const int ds = sx - sy;
    if (ds == 0) return 0; /* copying an equal strategy changes nothing */
    const int dsig = sig_x - sig_y;
    if (u < T[(dsig + 25) * 3 + (ds + 1)]) { /* Eq. (3) via the table */
        s[(size_t)i * L + j] = (uint8_t)sy;
        return sy ? +1 : -1;
    }
    return 0;
}

/* The elementary step of oracle A at site (i, j) of colour k in sweep t. */
static int elementary_step(uint8_t* s, int L, const uint32_t* T, uint64_t seed,
                           uint32_t t, int k, int i, int j)
{
    uint32_t w[4];
    philox_site(seed, (uint32_t)(i * L + j), t, (uint32_t)k, 0u, w);
    return imitate(s, L, T, i, j, (int)(w[0] >> 30), w[1]);
}

/* xorshift64* for the test hook that permutes the in-colour visiting order
 * (Vigna, "An experimental exploration of Marsaglia's xorshift generators").
 * It never touches the dynamics' random numbers. */
static uint64_t xs64(uint64_t* st)
{
    uint64_t x = *st;
    x ^= x >> 12; x ^= x << 25; x ^= x >> 27;
    *st = x;
    return x * 2685821657736338717ull;
}

/* Run n sweeps starting at absolute sweep index t0 on the lattice s (in
 * place).  counts[q] = N_C after sweep t0 + q (full recount, Eq. (4) sum).
 * order: 0 raster, 1 reversed raster, 2 random permutation (order_seed) of
 * the sites inside each colour class; the result must not depend on it. */
int pgg_ref_sweep(uint8_t* s, uint32_t L, double r, double K, uint64_t seed,
                  uint64_t t0, uint32_t n, uint64_t* counts, int order,
                  uint64_t order_seed)
{
    if (!valid_L(L) || t0 + (uint64_t)n > 4294967296ull || order < 0 || order > 2)
        return PGG_REF_EINVAL;
    uint32_t T[153];
    int rc = pgg_ref_table(r, K, T);
    if (rc) return rc;
    const uint32_t per = (L / 4) * (L / 4);
    uint32_t* perm = NULL;
    if (order == 2) {
        perm = (uint32_t*)malloc(sizeof(uint32_t) * per);
        if (!perm) return PGG_REF_ENOMEM;
    }
    uint64_t ost = order_seed | 1ull;
    for (uint32_t q = 0; q < n; ++q) {
        const uint32_t t = (uint32_t)(t0 + q);
        for (int k = 0; k < 16; ++k) {
            const int a = k / 4, b = k % 4;
            if (order == 2) {
                for (uint32_t m = 0; m < per; ++m) perm[m] = m;
                for (uint32_t m = per - 1; m > 0; --m) {
                    uint32_t z = (uint32_t)(xs64(&ost) % (uint64_t)(m + 1));
                    uint32_t tmp = perm[m]; perm[m] = perm[z]; perm[z] = tmp;
                }
            }
            for (uint32_t m = 0; m < per; ++m) {
                uint32_t idx = order == 0 ? m : order == 1 ? per - 1 - m : perm[m];
                int i = a + 4 * (int)(idx / (L / 4));
                int j = b + 4 * (int)(idx % (L / 4));
                elementary_step(s, (int)L, T, seed, t, k, i, j);
            }
        }
        if (counts) counts[q] = pgg_ref_count(s, L);
    }
    free(perm);
    return PGG_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Oracle C: the double tiling decomposition of Sec. IV (Fig. 2).  The       */
/* lattice is cut into 4 x 4 domains (I, J) = rows 4I..4I+3, columns         */
/* 4J..4J+3; rows of domains alternate the type sequences 1,2,1,2,... (I     */
/* even) and 3,4,3,4,... (I odd), so domain (I, J) has type                 */
/* 1 + 2 (I mod 2) + (J mod 2).  A full Monte Carlo step runs four parts,    */
/* types 1, 2, 3, 4 in turn; in a part every domain of that type performs    */
/* 16 elementary steps of Sec. III in random sequential order -- x uniform   */
/* among the domain's 16 players, y uniform among x's four neighbours (which */
/* may lie outside the domain) -- so each player gets one chance per MCS on  */
/* average.  Domains of one type neither share a player nor read each       */
/* other's players (they are 4 sites apart and a step reads at most 3 sites  */
/* beyond x), so a part's domains are independent.  L must be a multiple of  */
/* 8 (Sec. IV).                                                             */
/* Random numbers (our reading; the paper names no generator): step m of    */
/* part p in sweep t of domain (I, J) takes the Philox block of counter      */
/* (I * L/4 + J, t, 16 p + m, 2): x is player w0 >> 28 of the domain         */
/* (row-major, (w0 >> 28) / 4 rows down, (w0 >> 28) mod 4 columns right),    */
/* d = (w0 >> 26) mod 4 picks y as in oracle A, u = w1.                       */
/* ------------------------------------------------------------------------ */
static int tiled_step(uint8_t* s, int L, const uint32_t* T, uint64_t seed, uint32_t t,
                      int part, int m, int I, int J)
{
    uint32_t w[4];
    philox_site(seed, (uint32_t)(I * (L / 4) + J), t, (uint32_t)(16 * part + m), 2u, w);
    const int idx = (int)(w[0] >> 28);
    return imitate(s, L, T, 4 * I + idx / 4, 4 * J + idx % 4, (int)((w[0] >> 26) & 3u), w[1]);
}

/* n tiled Monte Carlo steps from absolute sweep index t0 (in place);
 * counts[q] = N_C after sweep t0 + q.  order: 0 raster, 1 reversed raster,
 * 2 random permutation (order_seed) of the domains inside each part; the
 * result must not depend on it. */
int pgg_ref_sweep_tiled(uint8_t* s, uint32_t L, double r, double K, uint64_t seed,
                        uint64_t t0, uint32_t n, uint64_t* counts, int order,
                        uint64_t order_seed)
{
    if (!valid_L(L) || (L % 8) != 0 || t0 + (uint64_t)n > 4294967296ull || order < 0 || order > 2)
        return PGG_REF_EINVAL;
    uint32_t T[153];
    int rc = pgg_ref_table(r, K, T);
    if (rc) return rc;
    const uint32_t half = L / 8;            /* domains of one type per row of domains */
    const uint32_t per = half * half;       /* domains of one type */
    uint32_t* perm = NULL;
    if (order == 2) {
        perm = (uint32_t*)malloc(sizeof(uint32_t) * per);
        if (!perm) return PGG_REF_ENOMEM;
    }
    uint64_t ost = order_seed | 1ull;
    for (uint32_t q = 0; q < n; ++q) {
        const uint32_t t = (uint32_t)(t0 + q);
        for (int part = 0; part < 4; ++part) {
            const int pi = part / 2, pj = part % 2;  /* type 1 + part: (I mod 2, J mod 2) */
            if (order == 2) {
                for (uint32_t m = 0; m < per; ++m) perm[m] = m;
                for (uint32_t m = per - 1; m > 0; --m) {
                    uint32_t z = (uint32_t)(xs64(&ost) % (uint64_t)(m + 1));
                    uint32_t tmp = perm[m]; perm[m] = perm[z]; perm[z] = tmp;
                }
            }
            for (uint32_t e = 0; e < per; ++e) {
                uint32_t idx = order == 0 ? e : order == 1 ? per - 1 - e : perm[e];
                int I = pi + 2 * (int)(idx / half);
                int J = pj + 2 * (int)(idx % half);
                for (int m = 0; m < 16; ++m) tiled_step(s, (int)L, T, seed, t, part, m, I, J);
            }
        }
        if (counts) counts[q] = pgg_ref_count(s, L);
    }
    free(perm);
    return PGG_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Oracle B: textbook random-sequential Monte Carlo (Sec. III).  One MCS is  */
/* L^2 elementary steps, each on a uniformly chosen player x, with y chosen  */
/* uniformly among its four nearest neighbours; payoffs from Eq. (1)-(2)     */
/* group by group; x copies y with the probability W of Eq. (3).             */
/* Random numbers: xoshiro256** seeded through splitmix64 (Blackman and      */
/* Vigna, "Scrambled linear pseudorandom number generators").               */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t s[4]; } xo256;

static uint64_t splitmix64(uint64_t* z)
{
    uint64_t v = (*z += 0x9E3779B97F4A7C15ull);
    v = (v ^ (v >> 30)) * 0xBF58476D1CE4E5B9ull;
    v = (v ^ (v >> 27)) * 0x94D049BB133111EBull;
    return v ^ (v >> 31);
}

static uint64_t rotl64(uint64_t v, int k) { return (v << k) | (v >> (64 - k)); }

static uint64_t xo_next(xo256* g)
{
    uint64_t* s = g->s;
    const uint64_t out = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return out;
}

/* uniform integer in [0, n) by rejection (no modulo bias) */
static uint64_t xo_below(xo256* g, uint64_t n)
{
    uint64_t lim = UINT64_MAX - (UINT64_MAX % n);
    uint64_t v;
    do { v = xo_next(g); } while (v >= lim);
    return v % n;
}

static double xo_unit(xo256* g) { return (double)(xo_next(g) >> 11) * 0x1.0p-53; }

int pgg_ref_rs_run(uint8_t* s, uint32_t L, double r, double K, uint64_t seed,
                   uint32_t n_mcs, uint64_t* counts)
{
    if (L < 3 || L > 32768 || !(isfinite(r) && r >= 0.0 && isfinite(K) && K > 0.0))
        return PGG_REF_EINVAL;
    xo256 g;
    uint64_t z = seed;
    for (int q = 0; q < 4; ++q) g.s[q] = splitmix64(&z);
    const uint64_t sites = (uint64_t)L * L;
    for (uint32_t mcs = 0; mcs < n_mcs; ++mcs) {
        for (uint64_t step = 0; step < sites; ++step) {
            const uint64_t x = xo_below(&g, sites);
            const int i = (int)(x / L), j = (int)(x % L);
            const int d = (int)xo_below(&g, 4);
            const int yi = wrap((int64_t)i + DIR_DI[d], (int)L);
            const int yj = wrap((int64_t)j + DIR_DJ[d], (int)L);
            const double u = xo_unit(&g);
            const uint8_t sx = s[x], sy = s[(size_t)yi * L + yj];
            if (sx == sy) continue;
            const double pi_x = pgg_ref_payoff(s, (int)L, r, i, j);
            const double pi_y = pgg_ref_payoff(s, (int)L, r, yi, yj);
            const double w = 1.0 / (1.0 + exp((pi_x - pi_y) / K)); /* Eq. (3) */
            if (u < w) s[x] = sy;
        }
        if (counts) counts[mcs] = pgg_ref_count(s, L);
    }
    return PGG_REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Oracle D: the pairwise prisoner's dilemma that Sec. VI names as the next  */
/* game for the same scheme: the game is played pairwise with each of the    */
/* four nearest neighbours instead of in groups, so an elementary step reads */
/* one line less in every direction (radius 2 around x instead of 3).        */
/* The paper gives no payoffs; our reading is the weak prisoner's dilemma    */
/* with temptation b: a cooperator meeting a cooperator earns R = 1, a       */
/* defector meeting a cooperator earns T = b, everything else earns 0        */
/* (S = P = 0).  A player's payoff is the sum of its four games, and the     */
/* imitation is the elementary step of Sec. III with the Fermi rule Eq. (3). */
/*                                                                          */
/* Schedule (our reading): with a radius-2 read set, sites 4 apart (L1) may  */
/* update together, and with L a multiple of 4 the densest such colouring    */
/* has 8 classes: the cosets of the sublattice spanned by (2, 2) and (4, 0). */
/* Site (i, j) has class k = 4 (i mod 2) + ((j - 2 h) mod 4) with h =         */
/* (i div 2) mod 2; a sweep runs k = 0..7 in ascending order, every site     */
/* once.  Random numbers: the Philox block of counter (x, t, k, 0), d = w0    */
/* >> 30 as in oracle A, u = w1; the initial state as in oracle A.           */
/* ------------------------------------------------------------------------ */

/* Payoff of the player at (i, j) literally from the four pairwise games,
 * binary64 (R = 1, T = b, S = P = 0). */
double pgg_ref_pd_payoff(const uint8_t* s, int L, double b, int i, int j)
{
    const double R = 1.0, Tm = b, S = 0.0, P = 0.0;
    const int sx = at(s, L, i, j);
    double total = 0.0;
    for (int d = 0; d < 4; ++d) {
        const int sy = at(s, L, (int64_t)i + DIR_DI[d], (int64_t)j + DIR_DJ[d]);
        total += sx ? (sy ? R : S) : (sy ? Tm : P);
    }
    return total;
}

/* Cooperators among the four nearest neighbours of (i, j), indexed modulo L
 * on every access.  With R = 1, T = b and S = P = 0 a cooperator earns
 * exactly this number n and a defector b n: the integer form the table uses. */
int pgg_ref_pd_ncoop(const uint8_t* s, int L, int i, int j)
{
    int n = 0;
    for (int d = 0; d < 4; ++d) n += at(s, L, (int64_t)i + DIR_DI[d], (int64_t)j + DIR_DJ[d]);
    return n;
}

/* T[(dir * 5 + n_x) * 5 + n_y]: dir 0 = x cooperates and y defects (Pi_x =
 * n_x, Pi_y = b n_y), dir 1 = x defects and y cooperates (Pi_x = b n_x, Pi_y =
 * n_y); W = 1 / (1 + exp((Pi_x - Pi_y) / K)) (Eq. (3)), stored as
 * min(2^32 - 1, floor(W * 2^32 + 1/2)).  The binary64 operation order is part
 * of the contract. */
int pgg_ref_pd_table(double b, double K, uint32_t* T)
{
    if (!(isfinite(b) && b >= 0.0 && isfinite(K) && K > 0.0)) return PGG_REF_EINVAL;
    for (int dir = 0; dir < 2; ++dir) {
        for (int nx = 0; nx <= 4; ++nx) {
            for (int ny = 0; ny <= 4; ++ny) {
                const double pix = dir == 0 ? 1.0 * (double)nx : b * (double)nx;
                const double piy = dir == 0 ? b * (double)ny : 1.0 * (double)ny;
                const double w = 1.0 / (1.0 + exp((pix - piy) / K));
                const double scaled = floor(w * 4294967296.0 + 0.5);
                T[(dir * 5 + nx) * 5 + ny] = scaled >= 4294967295.0 ? 4294967295u : (uint32_t)scaled;
            }
        }
    }
    return PGG_REF_OK;
}

/* Class of site (i, j) in the 8-colour schedule. */
int pgg_ref_pd_class(int i, int j)
{
    const int h = (i / 2) % 2;
    return 4 * (i % 2) + (((j - 2 * h) % 4) + 4) % 4;
}

/* One elementary step of the pairwise game at (i, j) of class k, sweep t. */
static int pd_step(uint8_t* s, int L, const uint32_t* T, uint64_t seed, uint32_t t, int k, int i, int j)
{
    uint32_t w[4];
    philox_site(seed, (uint32_t)(i * L + j), t, (uint32_t)k, 0u, w);
    const int d = (int)(w[0] >> 30);
    const int yi = wrap((int64_t)i + DIR_DI[d], L), yj = wrap((int64_t)j + DIR_DJ[d], L);
    const int sx = s[(size_t)i * L + j], sy = s[(size_t)yi * L + yj];
    if (sx == sy) return 0;
    const int nx = pgg_ref_pd_ncoop(s, L, i, j), ny = pgg_ref_pd_ncoop(s, L, yi, yj);
    const int dir = sx ? 0 : 1;
    if (w[1] < T[(dir * 5 + nx) * 5 + ny]) {
        s[(size_t)i * L + j] = (uint8_t)sy;
        return sy ? +1 : -1;
    }
    return 0;
}

/* n sweeps of the 8-colour schedule from absolute sweep index t0 (in
 * place); counts[q] = N_C after sweep t0 + q.  order as for oracle A. */
int pgg_ref_pd_sweep(uint8_t* s, uint32_t L, double b, double K, uint64_t seed,
                     uint64_t t0, uint32_t n, uint64_t* counts, int order, uint64_t order_seed)
{
    if (!valid_L(L) || t0 + (uint64_t)n > 4294967296ull || order < 0 || order > 2)
        return PGG_REF_EINVAL;
    uint32_t T[50];
    int rc = pgg_ref_pd_table(b, K, T);
    if (rc) return rc;
    /* the sites of one class, listed once */
    const uint32_t per = L * L / 8;
    uint32_t* cls = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)L * L);
    uint32_t* perm = (uint32_t*)malloc(sizeof(uint32_t) * per);
    if (!cls || !perm) { free(cls); free(perm); return PGG_REF_ENOMEM; }
    uint64_t ost = order_seed | 1ull;
    for (uint32_t q = 0; q < n; ++q) {
        const uint32_t t = (uint32_t)(t0 + q);
        for (int k = 0; k < 8; ++k) {
            uint32_t m = 0;
            for (uint32_t i = 0; i < L; ++i)
                for (uint32_t j = 0; j < L; ++j)
                    if (pgg_ref_pd_class((int)i, (int)j) == k) cls[m++] = i * L + j;
            for (uint32_t e = 0; e < per; ++e) perm[e] = order == 1 ? per - 1 - e : e;
            if (order == 2) {
                for (uint32_t e = per - 1; e > 0; --e) {
                    uint32_t z = (uint32_t)(xs64(&ost) % (uint64_t)(e + 1));
                    uint32_t tmp = perm[e]; perm[e] = perm[z]; perm[z] = tmp;
                }
            }
            for (uint32_t e = 0; e < per; ++e) {
                const uint32_t x = cls[perm[e]];
                pd_step(s, (int)L, T, seed, t, k, (int)(x / L), (int)(x % L));
            }
        }
        if (counts) counts[q] = pgg_ref_count(s, L);
    }
    free(cls);
    free(perm);
    return PGG_REF_OK;
}
