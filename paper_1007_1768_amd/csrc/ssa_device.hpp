// ssa_device.hpp -- per-lane arithmetic of the direct-method SSA on gfx950.
//
// Counter-based random numbers, the 53-bit uniforms, the exponential waiting time and the
// mass-action propensity, each written to the arithmetic contract stated in include/ssa.h
// (the paper fixes the semantics in Section 2 and Section 3.2, not the roundings).
// Binary64 throughout, compiled with -ffp-contract=off: every '*' and '+' below is one
// IEEE operation, and fused multiply-adds appear only where written as __builtin_fma.
#pragma once

#if !defined(__HIPCC_RTC__)
#include <hip/hip_runtime.h>
#include <stdint.h>
#else   // the run-time compiler provides the HIP device API and its own fixed-width types
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::uint64_t uint64_t;
typedef __hip_internal::int32_t int32_t;
typedef __hip_internal::int64_t int64_t;
typedef __hip_internal::uint64_t uintptr_t;
#endif

namespace ssa {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 4x32 S-box with
// the key bumped by the two Weyl increments between rounds.  The key is the seed, the
// same for every lane, so its schedule stays in scalar registers.
struct u32x4 { uint32_t v0, v1, v2, v3; };

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return u32x4{c0, c1, c2, c3};
}

// 53 high bits of the 64-bit word hi:lo as an exact binary64 integer (< 2^53):
// (hi >> 11) * 2^32 + ((hi << 21) | (lo >> 11)); both parts convert exactly and the sum is
// exact because it stays below 2^53.
__device__ __forceinline__ double top53(uint32_t lo, uint32_t hi) {
    const uint32_t up = hi >> 11;
    const uint32_t dn = (hi << 21) | (lo >> 11);
    return __builtin_fma((double)up, 4294967296.0, (double)dn);
}

// r1 in (0, 1]: (top53 + 1) 2^-53 (top53 + 1 <= 2^53 is exact).
__device__ __forceinline__ double uniform_open0(uint32_t lo, uint32_t hi) {
    return (top53(lo, hi) + 1.0) * 0x1p-53;
}
// r2 in [0, 1): top53 * 2^-53.
__device__ __forceinline__ double uniform_open1(uint32_t lo, uint32_t hi) {
    return top53(lo, hi) * 0x1p-53;
}

// -ln r for r in [2^-53, 1] from 2 atanh((m-1)/(m+1)):
//   r = m 2^E, m in (sqrt2/2, sqrt2];  f = (m-1)/(m+1);  s = f f;
//   P = C10, P = fma(P, s, Cn) for n = 9..1, Cn = 2/(2n+1) rounded once;
//   ln m = fma(f, s P, f + f);  ln r = fma(E, LN2_HI, fma(E, LN2_LO, ln m)).
// LN2_HI keeps 32 significant bits of ln 2, so E * LN2_HI is exact; LN2_LO is the rest.
// p s + c rounded once, as the three-operand VOP3 instruction: for a loop-invariant c the
// compiler otherwise copies c into the accumulator and uses the two-operand form, one more
// instruction per term.
__device__ __forceinline__ double fma3(double p, double s, double c) {
    double out;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(out) : "v"(p), "v"(s), "v"(c));
    return out;
}

__device__ __forceinline__ double neg_log(double r) {
    constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
    constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
    constexpr double kSqrt2 = 0x1.6a09e667f3bcdp+0;
    const uint64_t b = (uint64_t)__double_as_longlong(r);
    int E = (int)((b >> 52) & 0x7ff) - 1023;
    double m = __longlong_as_double((long long)((b & 0x000fffffffffffffull) | 0x3ff0000000000000ull));
    if (m > kSqrt2) {
        m = m * 0.5;
        E = E + 1;
    }
    const double f = (m - 1.0) / (m + 1.0);
    const double s = f * f;
    double P = 2.0 / 21.0;
    P = fma3(P, s, 2.0 / 19.0);
    P = fma3(P, s, 2.0 / 17.0);
    P = fma3(P, s, 2.0 / 15.0);
    P = fma3(P, s, 2.0 / 13.0);
    P = fma3(P, s, 2.0 / 11.0);
    P = fma3(P, s, 2.0 / 9.0);
    P = fma3(P, s, 2.0 / 7.0);
    P = fma3(P, s, 2.0 / 5.0);
    P = fma3(P, s, 2.0 / 3.0);
    const double t = s * P;
    const double lnm = __builtin_fma(f, t, f + f);
    const double Ed = (double)E;
    return -__builtin_fma(Ed, kLn2Hi, __builtin_fma(Ed, kLn2Lo, lnm));
}

}  // namespace ssa
