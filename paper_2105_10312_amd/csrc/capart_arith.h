// Integer arithmetic of the engine's kernels, written so that it also compiles
// as plain host C++ (define CAPART_HD empty) for exhaustive CPU checks.
#pragma once

#include <stdint.h>

#ifndef CAPART_HD
#define CAPART_HD __host__ __device__
#endif

namespace capart {

// Saturation value for execution times: larger than every admissible deadline
// (D < 2^31), so a saturated time compares exactly like the true one against
// D and T.
constexpr uint32_t C_SAT = 0x80000000u;
constexpr uint16_t MMIN_NONE = 0xFFFFu;

// c = ceil(2^64 / T) split in 32-bit halves, for T >= 2.
CAPART_HD inline void magic_u32(uint32_t T, uint32_t *clo, uint32_t *chi)
{
    uint64_t c = (T >= 2) ? (~0ull / T) + 1ull : 0ull;  // ceil(2^64/T) = floor((2^64-1)/T) + 1
    *clo = (uint32_t)c;
    *chi = (uint32_t)(c >> 32);
}

// floor(x / T) for any 32-bit x, from c = ceil(2^64/T): the high 64 bits of
// the 96-bit product c*x (the error term c*x/2^64 - x/T < x/2^64 <= 1/T keeps
// the floor exact).  Two 32-bit multiplies: mul_hi then a 64-bit mad.
CAPART_HD inline uint32_t floordiv_magic(uint32_t x, uint32_t clo, uint32_t chi)
{
    uint32_t lo_hi = (uint32_t)(((uint64_t)clo * x) >> 32);
    return (uint32_t)(((uint64_t)chi * x + lo_hi) >> 32);
}

// floor(x / T) for 0 <= x < 2^31 with a single 32-bit multiplier
// (Granlund and Montgomery 1994, Theorem 4.2, with N = 31 dividend bits):
// l = ceil(log2 T) and m = ceil(2^(31+l) / T) give m T - 2^(31+l) < T <= 2^l,
// so floor(x/T) = floor(m x / 2^(31+l)) = mul_hi(m, 2x) >> l; m < 2^32 (2^31
// when T is a power of two, T = 1 included).  One mul_hi and one shift.
CAPART_HD inline void magic31(uint32_t T, uint32_t *m, uint32_t *l)
{
    uint32_t s = 0;
    while (s < 31u && (1u << s) < T) s++;
    *m = (uint32_t)((((uint64_t)1 << (31u + s)) + T - 1u) / T);
    *l = s;
}

// The same m and l from c = ceil(2^64 / T) (magic_u32) without a division:
// ceil(c / 2^(33-l)) = ceil(2^(31+l) / T), since nested ceilings of
// divisions by positive integers compose; T = 1 (no c) gives 2^31 and 0.
CAPART_HD inline void magic31_of(uint32_t T, uint32_t clo, uint32_t chi, uint32_t *m, uint32_t *l)
{
    if (T < 2u) {
        *m = 0x80000000u;
        *l = 0u;
        return;
    }
    const uint32_t s = 32u - (uint32_t)__builtin_clz(T - 1u);  // ceil(log2 T), 1..31
    const uint64_t c = ((uint64_t)chi << 32) | clo;
    *m = (uint32_t)((c + (((uint64_t)1 << (33u - s)) - 1u)) >> (33u - s));
    *l = s;
}

// x2 = 2x for the x above.
CAPART_HD inline uint32_t floordiv31(uint32_t x2, uint32_t m, uint32_t l)
{
    return (uint32_t)(((uint64_t)m * x2) >> 32) >> l;
}

// Execution time on m units without conflict: C_seq + ceil(C_par / m).
// With C_seq + C_par < 2^31 the result is < 2^31.
CAPART_HD inline uint32_t time_n(uint32_t Cs, uint32_t Cp, uint32_t m)
{
    return Cs + (Cp + m - 1u) / m;
}

// Execution time in conflict: ceil(k * Cn / 1000), saturated at C_SAT.
CAPART_HD inline uint32_t time_c(uint32_t k, uint32_t cn)
{
    uint64_t x = (uint64_t)k * cn;  // < 2^20 * 2^31
    uint64_t c = (x + 999u) / 1000u;
    return c > C_SAT ? C_SAT : (uint32_t)c;
}

// ceil(C * 2^32 / T) - 1 for 1 <= C <= T (value in [0, 2^32 - 1]); all ones when
// C > T (the task cannot be in a feasible partition then).
CAPART_HD inline uint32_t util_q32_m1(uint32_t C, uint32_t T)
{
    if (C > T) return 0xFFFFFFFFu;
    uint64_t num = (uint64_t)C << 32;
    uint64_t q = (num + T - 1u) / T;
    return (uint32_t)(q - 1u);
}

// util_q32_m1 without a 64-bit division, from c = ceil(2^64/T) as split by
// magic_u32 (T >= 2): y = C*chi + mul_hi(C, clo) = floor(C*c / 2^32) exceeds
// v = C*2^32/T by less than C/2^32 < 1/2, so y is floor(v) or floor(v) + 1;
// one product y*T (< 2^64 since y <= 2^32 + 1 and T < 2^31) settles it.
CAPART_HD inline uint32_t util_q32_m1_magic(uint32_t C, uint32_t T, uint32_t clo, uint32_t chi)
{
    if (C > T) return 0xFFFFFFFFu;
    if (T == 1u) return 0xFFFFFFFFu;  // C = T = 1: 2^32 - 1
    const uint64_t num = (uint64_t)C << 32;
    uint64_t y = (uint64_t)C * chi + (uint32_t)(((uint64_t)C * clo) >> 32);
    if (y * T > num) y--;                   // now y = floor(v)
    const uint64_t q = y + (y * T != num);  // ceil(v)
    return (uint32_t)(q - 1u);
}

// floor(x / X) for any 32-bit x and X >= 1 (X = 1 has no 2^64 reciprocal).
CAPART_HD inline uint32_t udiv_magic(uint32_t x, uint32_t X, uint32_t lo, uint32_t hi)
{
    return X == 1u ? x : floordiv_magic(x, lo, hi);
}

// floor and ceil of C 2^32 / X for 1 <= C <= X < 2^31 without a 64-bit
// division (the same correction as util_q32_m1_magic); both <= 2^32.
CAPART_HD inline void q32_floor_ceil(uint32_t C, uint32_t X, uint32_t lo, uint32_t hi, uint64_t *fl, uint64_t *cl)
{
    const uint64_t num = (uint64_t)C << 32;
    if (X == 1u) {
        *fl = *cl = num;
        return;
    }
    uint64_t y = (uint64_t)C * hi + (uint32_t)(((uint64_t)C * lo) >> 32);
    if (y * X > num) y--;
    *fl = y;
    *cl = y + (y * X != num);
}

// Lemma 2 closed form: least m in [1, M] with C_seq + ceil(C_par/m) <= D.
CAPART_HD inline uint16_t m_min(uint32_t Cs, uint32_t Cp, uint32_t D, uint32_t M)
{
    if (Cp == 0u) return Cs <= D ? (uint16_t)1 : MMIN_NONE;
    if (D <= Cs) return MMIN_NONE;
    uint32_t slack = D - Cs;
    uint32_t m = (Cp + slack - 1u) / slack;  // Cp < 2^31, slack < 2^31
    return m <= M ? (uint16_t)m : MMIN_NONE;
}

}  // namespace capart
