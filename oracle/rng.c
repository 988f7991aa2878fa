/*
 * Oracle random numbers (test infrastructure only).
 *
 * The paper asks only that every level draws fresh, independent random
 * numbers and that the coarse path reuses the fine path's increments
 * (Sec. 5, paragraph after eq. (eq:Yldef)).  The generator is the
 * counter-based Philox4x32-10 of Salmon, Moraes, Dror and Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3" (SC'11), written here from that
 * publication: a 4x32-bit counter and a 2x32-bit key, ten rounds, each round
 * taking the two 32x32->64 products of counter words 0 and 2 with the round
 * multipliers, xoring the high halves with the other two counter words and
 * the key, and bumping the key by the Weyl constants between rounds.
 *
 * Counter layout (a reading; the paper is silent):
 *   word 0 = j, the block index along the path (4 words per block),
 *   word 1 = path index s mod 2^32,
 *   word 2 = level + 256 * (s >> 32),
 *   word 3 = stream id.
 * Key = (seed mod 2^32, seed >> 32).
 * A path that needs fewer than four numbers from a stream (total = 1 or 2)
 * shares one block with q = 4/total neighbouring paths instead of leaving
 * words unused: path s reads block (0, s/q, ...) from word (s mod q) * total,
 * with s/q in place of s in words 1 and 2.
 *
 * Uniforms: u = ((x >> 8) + 1/2) 2^-24, exactly representable and in (0,1).
 * Normals: Box--Muller on a pair (u1, u2): rho = sqrt(-2 ln u1),
 * z0 = rho cos(2 pi u2), z1 = rho sin(2 pi u2).
 *
 * Pins: raw words against an independent library implementation of the same
 * published generator, and statistical checks of uniforms and normals.
 */
#include <math.h>
#include "oracle.h"

/* Round multipliers and Weyl increments from the Philox publication. */
#define PHX_MUL_A 0xD2511F53u
#define PHX_MUL_B 0xCD9E8D57u
#define PHX_WEYL_A 0x9E3779B9u
#define PHX_WEYL_B 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHX_WEYL_A;
            k1 += PHX_WEYL_B;
        }
        uint64_t prod_a = (uint64_t)PHX_MUL_A * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)PHX_MUL_B * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(prod_b >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod_b;
        uint32_t y2 = (uint32_t)(prod_a >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

double orc_u01(uint32_t x)
{
    return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0);
}

void orc_box_muller(uint32_t a, uint32_t b, double *z0, double *z1)
{
    const double pi = 3.14159265358979323846;
    double u1 = orc_u01(a), u2 = orc_u01(b);
    double rho = sqrt(-2.0 * log(u1));
    *z0 = rho * cos(2.0 * pi * u2);
    *z1 = rho * sin(2.0 * pi * u2);
}

void orc_counter(uint32_t j, uint64_t s, int level, int stream, uint32_t ctr[4])
{
    ctr[0] = j;
    ctr[1] = (uint32_t)(s & 0xffffffffu);
    ctr[2] = (uint32_t)level + 256u * (uint32_t)(s >> 32);
    ctr[3] = (uint32_t)stream;
}

static void seed_key(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xffffffffu);
    key[1] = (uint32_t)(seed >> 32);
}

void orc_path_words(uint64_t seed, int level, uint64_t s, int stream,
                    uint32_t nblocks, uint32_t *out)
{
    uint32_t key[2], ctr[4];
    seed_key(seed, key);
    for (uint32_t j = 0; j < nblocks; ++j) {
        orc_counter(j, s, level, stream, ctr);
        orc_philox4x32_10(ctr, key, out + 4 * (size_t)j);
    }
}

/* dim = 1: block j gives z[4j..4j+3] from the word pairs (0,1) and (2,3).
 * dim = 2: block j gives steps 2j and 2j+1, each step one pair (Z1, Z2).  */
void orc_path_normals(uint64_t seed, int level, uint64_t s, int stream, int dim,
                      int nsteps, double *z)
{
    uint32_t key[2], ctr[4], w[4];
    seed_key(seed, key);
    int total = nsteps * dim;           /* normals needed */
    if (total > 0 && total < 4) {       /* shared block, see above */
        int q = 4 / total;
        orc_counter(0, s / (uint64_t)q, level, stream, ctr);
        orc_philox4x32_10(ctr, key, w);
        double zz[4];
        orc_box_muller(w[0], w[1], &zz[0], &zz[1]);
        orc_box_muller(w[2], w[3], &zz[2], &zz[3]);
        for (int i = 0; i < total; ++i) z[i] = zz[(int)(s % (uint64_t)q) * total + i];
        return;
    }
    int nblocks = (total + 3) / 4;
    for (int j = 0; j < nblocks; ++j) {
        orc_counter((uint32_t)j, s, level, stream, ctr);
        orc_philox4x32_10(ctr, key, w);
        double a, b, c, d;
        orc_box_muller(w[0], w[1], &a, &b);
        orc_box_muller(w[2], w[3], &c, &d);
        double zz[4] = {a, b, c, d};
        for (int q = 0; q < 4; ++q)
            if (4 * j + q < total) z[4 * j + q] = zz[q];
    }
}

void orc_path_uniforms(uint64_t seed, int level, uint64_t s, int stream,
                       int nsteps, double *u)
{
    uint32_t key[2], ctr[4], w[4];
    seed_key(seed, key);
    if (nsteps > 0 && nsteps < 4) {     /* shared block */
        int q = 4 / nsteps;
        orc_counter(0, s / (uint64_t)q, level, stream, ctr);
        orc_philox4x32_10(ctr, key, w);
        for (int i = 0; i < nsteps; ++i) u[i] = orc_u01(w[(int)(s % (uint64_t)q) * nsteps + i]);
        return;
    }
    int nblocks = (nsteps + 3) / 4;
    for (int j = 0; j < nblocks; ++j) {
        orc_counter((uint32_t)j, s, level, stream, ctr);
        orc_philox4x32_10(ctr, key, w);
        for (int q = 0; q < 4; ++q)
            if (4 * j + q < nsteps) u[4 * j + q] = orc_u01(w[q]);
    }
}
