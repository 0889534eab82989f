/*
 * Oracle noise: counter-based Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11, Sec. 4) driving
 * Box-Muller (Box & Muller 1958) in FP64.  This is the Gaussian draw of
 * Alg. 1 (samples from N(nu_m, Sigma_m)); the paper does not say which
 * generator it uses.
 *
 * Counter = (sample j, control step k, quad q, iteration m); key = 64-bit
 * seed split (low, high).  Each quad gives four 32-bit words -> four
 * uniforms u = ((w >> 8) + 1) * 2^-24 in (0, 1] -> two Box-Muller pairs.
 * Quads 0..3 give 16 normals, of which the first 14 are the 14 joints.
 * TEST INFRASTRUCTURE ONLY.
 */
#include <math.h>
#include "oracle.h"

/* Philox constants as published in the SC'11 paper */
static const uint32_t PH_M0 = 0xD2511F53u, PH_M1 = 0xCD9E8D57u;
static const uint32_t PH_W0 = 0x9E3779B9u, PH_W1 = 0xBB67AE85u;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PH_W0; k1 += PH_W1; }
        uint64_t p0 = (uint64_t)PH_M0 * (uint64_t)x[0];
        uint64_t p1 = (uint64_t)PH_M1 * (uint64_t)x[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x[1] ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x[3] ^ k1;
        uint32_t y3 = lo0;
        x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
    }
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = x[3];
}

static double or_uniform(uint32_t w) { return ((double)(w >> 8) + 1.0) * (1.0 / 16777216.0); }

void or_normals14(uint64_t seed, uint32_t j, uint32_t k, uint32_t m, double z[14])
{
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    double zz[16];
    for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t ctr[4] = {j, k, q, m};
        uint32_t w[4];
        or_philox4x32_10(ctr, key, w);
        for (int pr = 0; pr < 2; ++pr) {
            double u1 = or_uniform(w[2 * pr]), u2 = or_uniform(w[2 * pr + 1]);
            double rad = sqrt(-2.0 * log(u1));
            double ang = 2.0 * M_PI * u2;
            zz[4 * q + 2 * pr] = rad * cos(ang);
            zz[4 * q + 2 * pr + 1] = rad * sin(ang);
        }
    }
    for (int d = 0; d < 14; ++d) z[d] = zz[d];
}

/* exported helpers for tests: raw words and uniforms */
void oracle_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out) { or_philox4x32_10(ctr, key, out); }

void oracle_noise(uint64_t seed, int K, int H, int m, double *z /* K*H*14 */)
{
    for (int j = 0; j < K; ++j)
        for (int k = 0; k < H; ++k)
            or_normals14(seed, (uint32_t)j, (uint32_t)k, (uint32_t)m, z + ((long)j * H + k) * 14);
}
