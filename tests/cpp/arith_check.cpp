// Host-compiled check of the kernels' integer arithmetic (capart_arith.h)
// against plain 128-bit reference expressions.  Exit status 0 = all passed.
#define CAPART_HD
#include "capart_arith.h"

#include <cstdio>
#include <cstdint>
#include <random>

using namespace capart;
typedef unsigned __int128 u128;

static int fails = 0;
#define CHECK(c) do { if (!(c)) { if (fails++ < 10) std::printf("FAIL %s line %d\n", #c, __LINE__); } } while (0)

int main()
{
    std::mt19937_64 rng(12345);
    // floor division by the 2^64 reciprocal: all 32-bit x for a few divisors,
    // random pairs over the full range, and edge cases
    const uint32_t edge_T[] = {2, 3, 5, 7, 10, 1000, 65535, 65536, 65537, 999999, 1u << 30, (1u << 31) - 1,
                               (1u << 31) - 2, 0x7FFFFFFDu, 3u << 29};
    const uint32_t edge_x[] = {0, 1, 2, 0x7FFFFFFEu, 0x7FFFFFFFu, 0x80000000u, 0xFFFFFFFEu, 0xFFFFFFFFu};
    for (uint32_t T : edge_T) {
        uint32_t lo, hi;
        magic_u32(T, &lo, &hi);
        for (uint32_t x : edge_x) CHECK(floordiv_magic(x, lo, hi) == x / T);
        for (int t = 0; t < 200000; t++) {
            uint32_t x = (uint32_t)rng();
            CHECK(floordiv_magic(x, lo, hi) == x / T);
            uint32_t y = (uint32_t)(rng() % (4ull * T)) + (uint32_t)(rng() % 3) * T;  // near multiples
            CHECK(floordiv_magic(y, lo, hi) == y / T);
            uint32_t z = (uint32_t)((rng() % 1000) * (uint64_t)T % 0x100000000ull);
            if (z) CHECK(floordiv_magic(z - 1, lo, hi) == (z - 1) / T);
            CHECK(floordiv_magic(z, lo, hi) == z / T);
        }
    }
    for (uint32_t T = 2; T < 3000; T++) {
        uint32_t lo, hi;
        magic_u32(T, &lo, &hi);
        for (uint32_t x = 0; x < 40000; x += 7) CHECK(floordiv_magic(x, lo, hi) == x / T);
        for (int t = 0; t < 200; t++) { uint32_t x = (uint32_t)rng(); CHECK(floordiv_magic(x, lo, hi) == x / T); }
    }
    for (int t = 0; t < 2000000; t++) {
        uint32_t T = 2 + (uint32_t)(rng() % ((1u << 31) - 3));
        uint32_t lo, hi;
        magic_u32(T, &lo, &hi);
        uint32_t x = (uint32_t)rng();
        CHECK(floordiv_magic(x, lo, hi) == x / T);
    }
    // floor division of x < 2^31 by the 32-bit multiplier: all x below 40000
    // and every x near a multiple for small T, the edge divisors, T = 1 and
    // powers of two, random pairs over the full range
    auto d31 = [&](uint32_t x, uint32_t T) {
        uint32_t m, l, m2, l2, lo, hi;
        magic31(T, &m, &l);
        CHECK(floordiv31(x << 1, m, l) == x / T);
        magic_u32(T, &lo, &hi);
        magic31_of(T, lo, hi, &m2, &l2);  // the division-free form gives the same pair
        CHECK(m2 == m && l2 == l);
    };
    for (uint32_t T = 1; T < 3000; T++) {
        for (uint32_t x = 0; x < 40000; x += 3) d31(x, T);
        for (uint32_t q = 1; q < 2000; q++) {
            const uint64_t z = (uint64_t)q * T * 997u % 0x80000000ull;
            if (z) d31((uint32_t)z - 1, T);
            d31((uint32_t)z, T);
        }
        d31(0x7FFFFFFFu, T);
        d31(0x7FFFFFFEu, T);
    }
    for (uint32_t k = 0; k < 31; k++) {
        const uint32_t T = 1u << k;
        for (uint32_t x : {0u, 1u, T - 1u, T, T + 1u, 0x7FFFFFFFu, 0x7FFFFFFEu}) if (x < 0x80000000u) d31(x, T);
        for (int t = 0; t < 20000; t++) d31((uint32_t)rng() & 0x7FFFFFFFu, T);
        if (T > 2) for (int t = 0; t < 20000; t++) d31((uint32_t)rng() & 0x7FFFFFFFu, T - 1), d31((uint32_t)rng() & 0x7FFFFFFFu, T + 1);
    }
    for (uint32_t T : edge_T) {
        for (uint32_t x : edge_x) if (x < 0x80000000u) d31(x, T);
        for (int t = 0; t < 200000; t++) {
            d31((uint32_t)rng() & 0x7FFFFFFFu, T);
            const uint64_t z = (rng() % 1000) * (uint64_t)T % 0x80000000ull;
            if (z) d31((uint32_t)z - 1, T);
            d31((uint32_t)z, T);
        }
    }
    for (int t = 0; t < 4000000; t++) {
        const uint32_t T = 1 + (uint32_t)(rng() % ((1u << 31) - 1));
        d31((uint32_t)rng() & 0x7FFFFFFFu, T);
        const uint64_t z = (rng() % 64) * (uint64_t)T;
        if (z && z < 0x80000000ull) d31((uint32_t)z - 1, T), d31((uint32_t)z, T);
    }
    // execution times, utilisation, Lemma 2
    for (int t = 0; t < 2000000; t++) {
        uint32_t Cs = (uint32_t)(rng() % (1u << 30)), Cp = (uint32_t)(rng() % (1u << 30));
        if (t % 3 == 0) { Cs = (uint32_t)(rng() % 1000); Cp = (uint32_t)(rng() % 100000); }
        if (Cs + Cp == 0) Cp = 1;
        uint32_t m = 1 + (uint32_t)(rng() % 255);
        uint32_t k = 1000 + (uint32_t)(rng() % 999001);
        uint64_t cn_ref = (uint64_t)Cs + ((uint64_t)Cp + m - 1) / m;
        uint32_t cn = time_n(Cs, Cp, m);
        CHECK(cn == cn_ref);
        u128 cc_ref = ((u128)k * cn_ref + 999) / 1000;
        uint32_t cc = time_c(k, cn);
        CHECK(cc == (cc_ref > C_SAT ? C_SAT : (uint32_t)cc_ref));
        uint32_t T = 1 + (uint32_t)(rng() % ((1u << 31) - 1));
        if (t % 2) T = cn + (uint32_t)(rng() % 1000);
        if (T >= (1u << 31)) T = (1u << 31) - 1;
        uint32_t u = util_q32_m1(cn, T);
        {
            uint32_t lo, hi;
            magic_u32(T, &lo, &hi);
            CHECK(util_q32_m1_magic(cn, T, lo, hi) == u);
            const uint32_t C2 = 1 + (uint32_t)(rng() % T);  // 1 <= C <= T over the full range
            CHECK(util_q32_m1_magic(C2, T, lo, hi) == util_q32_m1(C2, T));
        }
        if (cn <= T) {
            u128 q = (((u128)cn << 32) + T - 1) / T;
            CHECK((u128)u + 1 == q);
        } else {
            CHECK(u == 0xFFFFFFFFu);
        }
        uint32_t D = 1 + (uint32_t)(rng() % ((1u << 31) - 1));
        if (t % 2) D = cn_ref < (1u << 31) ? (uint32_t)cn_ref + (uint32_t)(rng() % 3) : D;
        uint32_t M = 1 + (uint32_t)(rng() % 255);
        uint16_t mm = m_min(Cs, Cp, D, M);
        uint32_t want = MMIN_NONE;
        for (uint32_t q = 1; q <= M; q++) if ((uint64_t)Cs + ((uint64_t)Cp + q - 1) / q <= D) { want = q; break; }
        CHECK(mm == want);
    }
    // division-free utilisation: every C <= T for small T, the ends of the
    // range for large T, and T = 1
    for (uint32_t T = 1; T < 2000; T++) {
        uint32_t lo, hi;
        magic_u32(T, &lo, &hi);
        for (uint32_t C = 1; C <= T + 1; C++) CHECK(util_q32_m1_magic(C, T, lo, hi) == util_q32_m1(C, T));
    }
    for (uint32_t T : edge_T) {
        uint32_t lo, hi;
        magic_u32(T, &lo, &hi);
        for (uint32_t d = 0; d < 3000 && d < T; d++) {
            CHECK(util_q32_m1_magic(T - d, T, lo, hi) == util_q32_m1(T - d, T));
            CHECK(util_q32_m1_magic(1 + d, T, lo, hi) == util_q32_m1(1 + d, T));
        }
    }
    // floor and ceil of C 2^32 / X and floor(x / X) with X = 1 allowed: every
    // C <= X for small X, random C over the full range for random X
    auto q32_check = [&](uint32_t C, uint32_t X) {
        uint32_t lo, hi;
        magic_u32(X, &lo, &hi);
        uint64_t fl, cl;
        q32_floor_ceil(C, X, lo, hi, &fl, &cl);
        const u128 num = (u128)C << 32;
        CHECK((u128)fl == num / X);
        CHECK((u128)cl == (num + X - 1) / X);
    };
    for (uint32_t X = 1; X < 1500; X++)
        for (uint32_t C = 1; C <= X; C++) q32_check(C, X);
    for (int t = 0; t < 2000000; t++) {
        const uint32_t X = 1 + (uint32_t)(rng() % ((1u << 31) - 1));
        q32_check(1 + (uint32_t)(rng() % X), X);
        q32_check(X, X);
        uint32_t lo, hi;
        magic_u32(X, &lo, &hi);
        const uint32_t x = (uint32_t)rng();
        CHECK(udiv_magic(x, X, lo, hi) == x / X);
    }
    for (uint32_t x : edge_x) CHECK(udiv_magic(x, 1u, 0u, 0u) == x);
    std::printf("%s (%d failures)\n", fails ? "FAILED" : "OK", fails);
    return fails ? 1 : 0;
}
