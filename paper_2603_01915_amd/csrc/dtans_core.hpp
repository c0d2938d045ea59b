// Core dtANS arithmetic of the CSR-dtANS format, shared by the HIP kernels and
// the library's host-side decoder (which verifies loaded containers and lets
// the kernels' integer formulation be exercised on the CPU).
//
// Format constants (Sec. IV-D of Schaetzle, Pegolotti, Pueschel, "Fast
// Entropy Decoding for Sparse MVM on GPUs", 2026): word radix W = 2^32, table
// size K = 2^12, multiplicity cap M = 2^8, l = 8 symbols per segment unpacked
// from o = 3 words (K^8 = W^3), f = 2 conditional checks (M^8 = W^2).
//
// Stream semantics used throughout:
//  * unpack: the 96-bit number w1*2^64 + w2*2^32 + w3 holds slots i1..i8 as
//    consecutive 12-bit fields, i1 in the lowest bits;
//  * a segment is the four nonzeros (d0 v0 d1 v1 d2 v2 d3 v3): odd positions
//    index the value table, even positions the column-delta table;
//  * digit group g (g = 1: symbols 1-4, g = 2: symbols 5-8) is appended to the
//    decoder state (d, r) as the least significant mixed-radix digits, then
//    check g runs: if r >= W the word w_g is extracted from the state
//    (w_g = d mod W, d /= W, r /= W), else w_g is read from the stream; w3 is
//    always read from the stream (Alg. 3 with the check placement of the
//    worked example in Sec. IV-D);
//  * a lane's last segment performs no checks and no loads (Sec. IV-F).
//
// GPU table entry (one 64-bit word per slot, shared by both alphabets):
//   bits  0..29  column delta of the delta-table slot
//   bit   30     the value-table slot holds the escape symbol
//   bit   31     the delta-table slot holds the escape symbol
//   bits 32..47  delta slot:  (base - 1) | digit << 8
//   bits 48..63  value slot:  (base - 1) | digit << 8
// plus one value (float or double) per slot in a second array.  When every
// base of both tables is at most 255 ("direct" tables) the two metadata
// fields hold base | digit << 8 instead (unused slots: base 1).
#pragma once

#include <stdint.h>

#if defined(__HIPCC__) || defined(__HIP__)
#include <hip/hip_runtime.h>
#define DTANS_HD __host__ __device__ __forceinline__
#else
#define DTANS_HD inline
#endif

namespace dtans {

constexpr int kSlots = 4096;   // K
constexpr int kMaxBase = 256;  // M
constexpr int kWave = 64;      // lanes per wavefront (and per encoded wave)
constexpr uint32_t kDeltaLimit = 1u << 30;  // table deltas are below this
// First delta of a row (or of a lane that starts inside a row): the column
// itself (the paper's choice, mode 0) or, in mode 1, the column minus the row
// plus kFirstBias modulo 2^32, which a banded matrix keeps within the table
// (the decoder starts such a row at row - kFirstBias and adds the delta).
constexpr uint32_t kFirstBias = 1u << 29;
DTANS_HD uint32_t first_base(uint32_t mode, uint32_t row) { return mode ? row - kFirstBias : 0u; }

// unpack three words into the eight 12-bit slot indices i1..i8
DTANS_HD void unpack8(uint32_t w1, uint32_t w2, uint32_t w3, uint32_t s[8]) {
    s[0] = w3 & 0xfffu;
    s[1] = (w3 >> 12) & 0xfffu;
    s[2] = (w3 >> 24) | ((w2 & 0xfu) << 8);
    s[3] = (w2 >> 4) & 0xfffu;
    s[4] = (w2 >> 16) & 0xfffu;
    s[5] = (w2 >> 28) | ((w1 & 0xffu) << 4);
    s[6] = (w1 >> 8) & 0xfffu;
    s[7] = w1 >> 20;
}

// inverse of unpack8
DTANS_HD void pack8(const uint32_t s[8], uint32_t &w1, uint32_t &w2, uint32_t &w3) {
    w3 = s[0] | (s[1] << 12) | (s[2] << 24);
    w2 = (s[2] >> 8) | (s[3] << 4) | (s[4] << 16) | (s[5] << 28);
    w1 = (s[5] >> 4) | (s[6] << 8) | (s[7] << 20);
}

// 16-bit slot metadata: (base - 1) | digit << 8
DTANS_HD uint32_t meta_base(uint32_t meta) { return (meta & 0xffu) + 1u; }
DTANS_HD uint32_t meta_digit(uint32_t meta) { return (meta >> 8) & 0xffu; }

// Accumulate one digit group of four symbols (meta of symbols 1..4 of the
// group, in stream order) into D (the group's digits as one mixed-radix
// number, first symbol most significant) and Rm1 = (product of bases) - 1,
// computed modulo 2^32 (the product is at most 2^32, which wraps to 0 and
// gives Rm1 = 2^32 - 1).
DTANS_HD void group4(uint32_t m0, uint32_t m1, uint32_t m2, uint32_t m3, uint32_t &D,
                     uint32_t &Rm1) {
    const uint32_t b1 = meta_base(m1), b2 = meta_base(m2), b3 = meta_base(m3);
    const uint32_t b23 = b2 * b3;                // <= 2^16
    const uint32_t lo = meta_digit(m2) * b3 + meta_digit(m3);  // < b2*b3
    const uint32_t hi = meta_digit(m0) * b1 + meta_digit(m1);  // < b0*b1
    D = hi * b23 + lo;                           // < 2^32
    const uint32_t b01 = meta_base(m0) * b1;     // <= 2^16
    Rm1 = b01 * b23 - 1u;                        // wraps exactly when the product is 2^32
}

// Append a digit group (D, R = Rm1 + 1) to the state (d, r), r < 2^32, and
// run the check.  Returns true when the word is extracted from the state
// (then *word is it); false when the caller must read it from the stream.
DTANS_HD bool append_and_check(uint32_t &d, uint32_t &r, uint32_t D, uint32_t Rm1,
                               uint32_t &word) {
    const uint64_t r64 = (uint64_t)r * Rm1 + r;              // r * R, < 2^64
    const uint64_t d64 = (uint64_t)d * Rm1 + ((uint64_t)d + D);  // d * R + D
    const bool extract = (r64 >> 32) != 0;
    if (extract) {
        word = (uint32_t)d64;
        d = (uint32_t)(d64 >> 32);
        r = (uint32_t)(r64 >> 32);
    } else {
        d = (uint32_t)d64;
        r = (uint32_t)r64;
    }
    return extract;
}

// The same two steps for tables whose bases are all at most 255 (an encoder
// multiplicity cap of 255 instead of M = 256): the GPU entry then holds the
// base itself in the low byte of a slot's metadata (base | digit << 8), so
// no +1 is needed, and R = product of the bases < 2^32 needs no wrap.
DTANS_HD void group4_direct(uint32_t m0, uint32_t m1, uint32_t m2, uint32_t m3, uint32_t &D,
                            uint32_t &R) {
    const uint32_t b1 = m1 & 0xffu, b2 = m2 & 0xffu, b3 = m3 & 0xffu;
    const uint32_t b23 = b2 * b3;
    const uint32_t lo = meta_digit(m2) * b3 + meta_digit(m3);
    const uint32_t hi = meta_digit(m0) * b1 + meta_digit(m1);
    D = hi * b23 + lo;
    R = (m0 & 0xffu) * b1 * b23;
}

#if defined(__HIPCC__) || defined(__HIP__)
// group4_direct from the high words of the four symbols' table entries
// (delta symbols 1 and 3 hold base | digit << 8 in bits 0..15, value symbols
// 2 and 4 in bits 16..31), on packed 16-bit lanes: v_perm gathers the bytes
// into (u16, u16) pairs, one packed multiply-add forms both two-digit parts
// and one packed multiply both two-base products, and a dot product joins
// them.  Same D and R as group4_direct (all intermediate values < 2^16).
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void group4_packed(uint32_t h0, uint32_t h1, uint32_t h2, uint32_t h3,
                                              uint32_t &D, uint32_t &R) {
    const uint32_t P = __builtin_amdgcn_perm(h3, h1, 0x0c060c02u);  // (b1, b3)
    const uint32_t Q = __builtin_amdgcn_perm(h2, h0, 0x0c050c01u);  // (d0, d2)
    const uint32_t S = __builtin_amdgcn_perm(h3, h1, 0x0c070c03u);  // (d1, d3)
    const uint32_t B = __builtin_amdgcn_perm(h2, h0, 0x0c040c00u);  // (b0, b2)
    const u16x2 T = __builtin_bit_cast(u16x2, Q) * __builtin_bit_cast(u16x2, P) +
                    __builtin_bit_cast(u16x2, S);                     // (d0 b1 + d1, d2 b3 + d3)
    const u16x2 U = __builtin_bit_cast(u16x2, B) * __builtin_bit_cast(u16x2, P);  // (b0 b1, b2 b3)
    const uint32_t V = __builtin_amdgcn_perm(1u, __builtin_bit_cast(uint32_t, U), 0x0c040302u);  // (b2 b3, 1)
    D = __builtin_amdgcn_udot2(T, __builtin_bit_cast(u16x2, V), 0u, false);
    R = __umul24((uint32_t)U.x, (uint32_t)U.y);
    // R < 2^32 is used as a 32-bit factor of the 64-bit state products; the
    // empty asm keeps the compiler from widening it to a 48-bit product
    // (which would double the 64-bit multiplies of append_direct)
    asm("" : "+v"(R));
}
#endif

DTANS_HD bool append_direct(uint32_t &d, uint32_t &r, uint32_t D, uint32_t R, uint32_t &word) {
    const uint64_t r64 = (uint64_t)r * R;
    const uint64_t d64 = (uint64_t)d * R + D;
    const bool extract = (r64 >> 32) != 0;
    if (extract) {
        word = (uint32_t)d64;
        d = (uint32_t)(d64 >> 32);
        r = (uint32_t)(r64 >> 32);
    } else {
        d = (uint32_t)d64;
        r = (uint32_t)r64;
    }
    return extract;
}

}  // namespace dtans
