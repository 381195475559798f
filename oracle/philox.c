/*
 * Oracle (test infrastructure only): the probe block X of the randomized SVD
 * (Alg. 3 samples the operator with independent random vectors).  The
 * normals come from the counter-based Philox4x64-10 generator written from
 * its published definition (Salmon, Moraes, Dror & Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11) and the Box-Muller transform.
 *
 * Entry (row, col) of X: counter (row / 4, col, 0, 0), key (seed, 0); the four
 * 64-bit outputs x_0..x_3 give u_i = ((x_i >> 11) + 1) 2^-53 in (0, 1] and
 *   row%4 == 0: sqrt(-2 ln u_0) cos(2 pi u_1)     row%4 == 1: ... sin(2 pi u_1)
 *   row%4 == 2: sqrt(-2 ln u_2) cos(2 pi u_3)     row%4 == 3: ... sin(2 pi u_3)
 * all in float64.
 */
#include <math.h>
#include <stdint.h>

#define PH_M0 0xD2E7470EE14C6C93ULL
#define PH_M1 0xCA5A826395121157ULL
#define PH_W0 0x9E3779B97F4A7C15ULL
#define PH_W1 0xBB67AE8584CAA73BULL

static void mulhilo(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void oracle_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PH_W0; k1 += PH_W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo(PH_M0, c0, &hi0, &lo0);
        mulhilo(PH_M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double unit_open0(uint64_t x) { return (double)((x >> 11) + 1) * 0x1.0p-53; }

double oracle_normal_entry(uint64_t seed, int64_t row, int64_t col) {
    uint64_t ctr[4] = {(uint64_t)(row / 4), (uint64_t)col, 0, 0};
    uint64_t key[2] = {seed, 0};
    uint64_t x[4];
    oracle_philox4x64_10(ctr, key, x);
    const double two_pi = 6.283185307179586476925286766559;
    int t = (int)(row % 4);
    double u_r = unit_open0(x[t < 2 ? 0 : 2]);
    double u_a = unit_open0(x[t < 2 ? 1 : 3]);
    double rad = sqrt(-2.0 * log(u_r));
    double ang = two_pi * u_a;
    return (t % 2 == 0) ? rad * cos(ang) : rad * sin(ang);
}

/* Column-major n x ncols block, leading dimension n. */
void oracle_normal_block(int64_t n, int32_t ncols, uint64_t seed, double* out) {
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ncols; ++j)
        for (int64_t r = 0; r < n; ++r) out[(int64_t)j * n + r] = oracle_normal_entry(seed, r, j);
}
