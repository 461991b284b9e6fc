/*
 * rng.c -- oracle randomness.  TEST INFRASTRUCTURE ONLY (see msst_oracle.h).
 *
 * The paper draws uniform numbers xi for free flights and phase sampling
 * (Sec. 3.1) and Gaussian z, epsilon for the CVAE prior and decoder posterior
 * (Sec. 3.2, Sec. 4.2) but names no generator.  Both sides of this project
 * use the counter-based Philox4x32-10 of Salmon et al. (SC'11), written here
 * from that publication: ten rounds of two 32x32->64 multiplications, the
 * key bumped by the two Weyl constants between rounds.
 */
#include "msst_oracle.h"

#include <math.h>

/* Multipliers and Weyl key increments published with Philox4x32. */
#define OR_PHILOX_MUL0 0xD2511F53u
#define OR_PHILOX_MUL1 0xCD9E8D57u
#define OR_PHILOX_WEYL0 0x9E3779B9u
#define OR_PHILOX_WEYL1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += OR_PHILOX_WEYL0;
            k1 += OR_PHILOX_WEYL1;
        }
        uint64_t prod0 = (uint64_t)OR_PHILOX_MUL0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)OR_PHILOX_MUL1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ x1 ^ k0;
        uint32_t n2 = hi0 ^ x3 ^ k1;
        x0 = n0;
        x1 = lo1;
        x2 = n2;
        x3 = lo0;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

static void or_block(uint64_t seed, uint32_t tag, uint64_t id, uint32_t c0, uint32_t out[4]) {
    uint32_t ctr[4] = {c0, (uint32_t)id, (uint32_t)(id >> 32), tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    or_philox4x32_10(ctr, key, out);
}

void or_philox_blocks(uint64_t seed, uint32_t tag, uint64_t id, uint32_t c0, int n, uint32_t* out) {
    for (int j = 0; j < n; ++j) or_block(seed, tag, id, c0 + (uint32_t)j, out + 4 * j);
}

/* Uniform on (0, 1]: the top 24 bits plus one, times 2^-24.  Every value is
 * exactly representable in binary32 and binary64, so both precisions see the
 * same number; 1 - xi of the paper's flight formula is this value itself. */
double or_u01(uint32_t word) { return ((double)(word >> 8) + 1.0) * (1.0 / 16777216.0); }

void or_uniform4(uint64_t seed, uint32_t tag, uint64_t id, uint32_t c0, double u[4]) {
    uint32_t w[4];
    or_block(seed, tag, id, c0, w);
    for (int i = 0; i < 4; ++i) u[i] = or_u01(w[i]);
}

/* Box-Muller: (u0, u1) -> (r cos 2 pi u1, r sin 2 pi u1), r = sqrt(-2 ln u0);
 * likewise (u2, u3). */
void or_normal4(uint64_t seed, uint32_t tag, uint64_t id, uint32_t c0, double nrm[4]) {
    double u[4];
    or_uniform4(seed, tag, id, c0, u);
    const double two_pi = 6.283185307179586476925286766559;
    double r0 = sqrt(-2.0 * log(u[0]));
    double r1 = sqrt(-2.0 * log(u[2]));
    nrm[0] = r0 * cos(two_pi * u[1]);
    nrm[1] = r0 * sin(two_pi * u[1]);
    nrm[2] = r1 * cos(two_pi * u[3]);
    nrm[3] = r1 * sin(two_pi * u[3]);
}
