/* Test helper: brute force over every state of the 18 sites that the payoffs
 * of a player x and its neighbour y depend on (the two radius-2 diamonds),
 * in all four directions, on an 8 x 8 periodic lattice.  For each state it
 * checks, through the oracle's exported functions, that the literal group-by-
 * group payoff of Eq. (1)-(2) equals (r/5)*sigma - 5*s for both players, and
 * that Pi_x - Pi_y = (r/5)*dSigma - 5*ds.  Prints the realised dSigma range
 * per ds and the number of failures. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

double pgg_ref_payoff(const uint8_t* s, int L, double r, int i, int j);
int pgg_ref_sigma(const uint8_t* s, int L, int i, int j);

int main(void) {
    const int L = 8, xi = 3, xj = 3;
    const int DI[4] = {0, 0, 1, -1}, DJ[4] = {1, -1, 0, 0};
    const double rs[3] = {3.8, 4.37, 1.5};
    long failures = 0, cases = 0;
    int lo[3] = {99, 99, 99}, hi[3] = {-99, -99, -99};
    for (int d = 0; d < 4; ++d) {
        int yi = xi + DI[d], yj = xj + DJ[d];
        int si[32], sj[32], n = 0;
        for (int i = 0; i < L; ++i)
            for (int j = 0; j < L; ++j) {
                int dx = abs(i - xi) + abs(j - xj), dy = abs(i - yi) + abs(j - yj);
                if (dx <= 2 || dy <= 2) { si[n] = i; sj[n] = j; ++n; }
            }
        if (n != 18) { printf("unexpected support %d\n", n); return 2; }
        uint8_t s[64];
        for (uint32_t m = 0; m < (1u << 18); ++m) {
            for (int q = 0; q < 64; ++q) s[q] = 0;
            for (int q = 0; q < 18; ++q) s[si[q] * L + sj[q]] = (m >> q) & 1u;
            int sgx = pgg_ref_sigma(s, L, xi, xj), sgy = pgg_ref_sigma(s, L, yi, yj);
            int sx = s[xi * L + xj], sy = s[yi * L + yj];
            int ds = sx - sy, dsig = sgx - sgy;
            if (dsig < lo[ds + 1]) lo[ds + 1] = dsig;
            if (dsig > hi[ds + 1]) hi[ds + 1] = dsig;
            for (int q = 0; q < 3; ++q) {
                double r = rs[q];
                double px = pgg_ref_payoff(s, L, r, xi, xj), py = pgg_ref_payoff(s, L, r, yi, yj);
                double ix = r * sgx / 5.0 - 5.0 * sx, iy = r * sgy / 5.0 - 5.0 * sy;
                double dint = r * dsig / 5.0 - 5.0 * ds;
                ++cases;
                if (fabs(px - ix) > 1e-9 || fabs(py - iy) > 1e-9 || fabs((px - py) - dint) > 1e-9)
                    ++failures;
            }
        }
    }
    printf("cases %ld failures %ld\n", cases, failures);
    for (int q = 0; q < 3; ++q) printf("ds %d dsig %d %d\n", q - 1, lo[q], hi[q]);
    return 0;
}
