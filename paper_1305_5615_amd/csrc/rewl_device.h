// rewl_device.h -- device building blocks of the REWL kernels (gfx950).
//
// Compiled with -ffp-contract=off: every floating-point expression below is a
// sequence of single IEEE binary64 operations rounded to nearest, so results
// are reproducible on any IEEE machine that evaluates the same operations.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rewl {

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications by the round multipliers on counter words 0 and 2,
// the high halves XOR-ed into the other two words and the round key, the key
// bumped by the Weyl constants after every round.
struct U4 {
    uint32_t x, y, z, w;
};

// rounds r0 .. r1-1 of Philox4x32-10 on (c, k); k is the key of round r0
__device__ __forceinline__ void philox_rounds(U4 &c, uint32_t &k0, uint32_t &k1, int r0, int r1)
{
    for (int r = r0; r < r1; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        // three-input XOR in one instruction (bitop3 truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96);
        c.y = (uint32_t)p1;
        c.w = (uint32_t)p0;
        c.x = n0;
        c.z = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1)
{
    U4 c{c0, c1, c2, c3};
#pragma unroll
    for (int r = 0; r < 10; ++r) philox_rounds(c, k0, k1, r, r + 1);
    return c;
}

// uniform integer in [0, n) from one word
__device__ __forceinline__ uint32_t mulhi32(uint32_t word, uint32_t n)
{
    return (uint32_t)(((uint64_t)word * n) >> 32);
}

// ln u for u = (2k+1) 2^-53, k = (hi << 20) | (lo >> 12): the odd integer
// n = 2k+1 < 2^53 is written as f 2^msb with f in [1, 2) directly from its
// bits, f is folded into [sqrt2/2, sqrt2], and ln f = 2 atanh(s) with
// s = (f-1)/(f+1) is summed as 2 (s + s z Q(z)), z = s^2,
// Q(z) = 1/3 + z/5 + ... + z^10/23 (coefficients RN(1/(2i+1)), Horner with
// fused multiply-adds).  ln 2 enters
// split as LN2_HI (32 fractional bits, so e * LN2_HI is exact) + LN2_LO.
// Two halves, so that a caller can interleave them with other work:
// ln_u_reduce gives s, z = s^2 and the exponent e, ln_u_sum the result.
struct LnU {
    double s, z;
    int e;
};

__device__ __forceinline__ LnU ln_u_reduce(uint32_t hi, uint32_t lo)
{
    const double kSqrt2 = 0x1.6a09e667f3bcdp+0;
    const uint64_t n = ((((uint64_t)hi << 20) | (uint64_t)(lo >> 12)) << 1) | 1u;
    const int msb = 63 - __clzll((long long)n);
    const uint64_t mant = (n << (52 - msb)) & 0x000FFFFFFFFFFFFFull;
    double f = __longlong_as_double((long long)(mant | 0x3FF0000000000000ull));
    int e = msb - 53;
    if (f > kSqrt2) {
        f = f * 0.5;
        e = e + 1;
    }
    LnU r;
    r.s = (f - 1.0) / (f + 1.0);
    r.z = r.s * r.s;
    r.e = e;
    return r;
}

// second half: e ln 2 + 2 (s + s z Q(z))
__device__ __forceinline__ double ln_u_sum(const LnU &a)
{
    const double kLn2Hi = 0x1.62e42ffp-1;
    const double kLn2Lo = -0x1.718432a1b0e26p-35;
    const double z = a.z, s = a.s;
    // Horner, each step one fused multiply-add (a single rounding)
    double Q = 1.0 / 23.0;
    Q = __fma_rn(Q, z, 1.0 / 21.0);
    Q = __fma_rn(Q, z, 1.0 / 19.0);
    Q = __fma_rn(Q, z, 1.0 / 17.0);
    Q = __fma_rn(Q, z, 1.0 / 15.0);
    Q = __fma_rn(Q, z, 1.0 / 13.0);
    Q = __fma_rn(Q, z, 1.0 / 11.0);
    Q = __fma_rn(Q, z, 1.0 / 9.0);
    Q = __fma_rn(Q, z, 1.0 / 7.0);
    Q = __fma_rn(Q, z, 1.0 / 5.0);
    Q = __fma_rn(Q, z, 1.0 / 3.0);
    const double ed = (double)a.e;
    const double lnf = (s + s * (z * Q)) * 2.0;
    return ed * kLn2Hi + (ed * kLn2Lo + lnf);
}

__device__ __forceinline__ double ln_u(uint32_t hi, uint32_t lo)
{
    return ln_u_sum(ln_u_reduce(hi, lo));
}

// Neighbours of site i = r L + c on the L x L torus; the row is
// mulhi(i, ceil(2^32 / L)), exact for i < 2^16 and L <= 256.
struct Nbrs {
    int rt, lf, dn, up, fw, bk;  // +x, -x, +y, -y (+z, -z on the L^3 torus)
};

__device__ __forceinline__ Nbrs neighbours(int i, int L, int N, uint32_t l_magic)
{
    const int r = (int)__umulhi((uint32_t)i, l_magic);
    const int c = i - r * L;
    Nbrs n;
    n.rt = (c + 1 == L) ? i - c : i + 1;
    n.lf = (c == 0) ? i + L - 1 : i - 1;
    n.dn = (r + 1 == L) ? c : i + L;
    n.up = (r == 0) ? i + N - L : i - L;
    n.fw = i;
    n.bk = i;
    return n;
}

// Neighbours of site i = (z L + y) L + x on the L x L x L torus, N = L^3;
// z = mulhi(i, ceil(2^32 / L^2)) and y likewise from the remainder, exact for
// i < 2^16.
__device__ __forceinline__ Nbrs neighbours3(int i, int L, int N, uint32_t l_magic,
                                            uint32_t l2_magic)
{
    const int L2 = L * L;
    const int z = (int)__umulhi((uint32_t)i, l2_magic);
    const int rem = i - z * L2;
    const int y = (int)__umulhi((uint32_t)rem, l_magic);
    const int x = rem - y * L;
    Nbrs n;
    n.rt = (x + 1 == L) ? i - x : i + 1;
    n.lf = (x == 0) ? i + L - 1 : i - 1;
    n.dn = (y + 1 == L) ? i - y * L : i + L;
    n.up = (y == 0) ? i + L2 - L : i - L;
    n.fw = (z + 1 == L) ? i - z * L2 : i + L2;
    n.bk = (z == 0) ? i + N - L2 : i - L2;
    return n;
}

}  // namespace rewl
