// Device-side building blocks shared by the sweep kernels: the Philox4x32-10
// block function, periodic index helpers and the payoff-sum stencil on
// bit-packed rows.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pgg {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each round forms the
// full 64-bit products of counter words 0 and 2 with two fixed odd
// multipliers; the new state is (hi(B*c2) ^ c1 ^ k0, lo(B*c2),
// hi(A*c0) ^ c3 ^ k1, lo(A*c0)), and the key advances by two Weyl constants.
constexpr uint32_t kPhiloxA = 0xD2511F53u;
constexpr uint32_t kPhiloxB = 0xCD9E8D57u;
constexpr uint32_t kWeylA = 0x9E3779B9u;
constexpr uint32_t kWeylB = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)kPhiloxA * c.x;
        const uint64_t pb = (uint64_t)kPhiloxB * c.z;
        c = make_uint4((uint32_t)(pb >> 32) ^ c.y ^ k0, (uint32_t)pb,
                       (uint32_t)(pa >> 32) ^ c.w ^ k1, (uint32_t)pa);
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return c;
}

// a ^ b ^ c in one VALU instruction: gfx950's three-input bitwise op with
// truth table 0x96 (c: a wave-uniform value in an SGPR).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// Words 0 and 1 of the Philox4x32-10 block of counter (c0, c1, c2, c3): the
// same rounds as philox4x32_10, with the three-input XORs as v_xor3_b32.
__device__ __forceinline__ uint2 philox4x32_10_w01(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                   uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 9; ++round) {
        const uint64_t pa = (uint64_t)kPhiloxA * c0;
        const uint64_t pb = (uint64_t)kPhiloxB * c2;
        const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(pa >> 32), c3, k1);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    const uint64_t pb = (uint64_t)kPhiloxB * c2;  // round 10: only words 0 and 1
    return make_uint2(xor3((uint32_t)(pb >> 32), c1, k0), (uint32_t)pb);
}

// (i + di) mod L for |di| <= 3 < L + 1, i in [0, L).
__device__ __forceinline__ int wrap_add(int i, int di, int L) {
    int v = i + di;
    v += (v < 0) ? L : 0;
    v -= (v >= L) ? L : 0;
    return v;
}

// Neighbour direction d = w0 >> 30: 0 E (j+1), 1 W (j-1), 2 S (i+1), 3 N (i-1).
__device__ __forceinline__ int dir_di(int d) { return (d == 2) - (d == 3); }
__device__ __forceinline__ int dir_dj(int d) { return (d == 0) - (d == 1); }

// Funnel shift: bits [sh, sh + 32) of the 64-bit value hi:lo.
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, int sh) {
    return __builtin_amdgcn_alignbit(hi, lo, (uint32_t)sh);
}

// 32 consecutive sites of a bit-packed row, columns c, c+1, ..., c+31 taken
// modulo L, returned with column c in bit 0.  `row` holds the L sites in
// ceil(L/32) words followed by at least one readable word; bits at columns
// >= L must be zero.  c may be in [-32, L).
__device__ __forceinline__ uint32_t row_window(const uint32_t* row, int L, int c) {
    while (c < 0) c += L;
    if (c + 32 <= L) {
        const int w = c >> 5;
        return funnel(row[w + 1], row[w], c & 31);
    }
    // The window crosses the periodic seam (or L < 32): assemble it from
    // pieces that each end at column L - 1.
    uint32_t out = 0;
    int got = 0;
    while (got < 32) {
        const int take = min(32 - got, L - c);
        const int w = c >> 5;
        uint32_t piece = funnel(row[w + 1], row[w], c & 31);
        if (take < 32) piece &= (1u << take) - 1u;
        out |= piece << got;
        got += take;
        c = 0;
    }
    return out;
}

// Sigma at a centre whose column sits at bit p (2 <= p <= 29) of five row
// windows a2 (row -2), a1 (row -1), b (row 0), c1 (row +1), c2 (row +2).
// Sigma = sum over the five groups containing the centre of their cooperator
// counts = 5 s_0 + 2 (nearest neighbours) + 2 (diagonals) + (axis, distance 2).
__device__ __forceinline__ int sigma_bits(uint32_t a2, uint32_t a1, uint32_t b, uint32_t c1,
                                          uint32_t c2, int p) {
    const uint32_t m_ends = 0x11u << (p - 2);  // columns p-2, p+2: weight 1
    const uint32_t m_near = 0x0Au << (p - 2);  // columns p-1, p+1: weight 2
    const uint32_t m_mid = 1u << p;            // column p
    const uint32_t m_three = 0x0Eu << (p - 2); // columns p-1..p+1
    const int ones = __popc(b & m_ends) + __popc(a2 & m_mid) + __popc(c2 & m_mid);
    const int twos = __popc(b & m_near) + __popc(a1 & m_three) + __popc(c1 & m_three);
    const int fives = __popc(b & m_mid);
    return ones + 2 * twos + 5 * fives;
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b to XCD
// b mod 8), each with its own L2.  This bijection of [0, n) makes XCD x run
// a contiguous range of logical blocks: x * (n / 8) + min(x, n mod 8) + b / 8.
__device__ __forceinline__ int xcd_major(int b, int n) {
    const int x = b & 7, k = b >> 3;
    const int q = n >> 3, rem = n & 7;
    return x * q + min(x, rem) + k;
}

}  // namespace pgg
