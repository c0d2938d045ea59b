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
// Device tables: see "Device tables of the HIP kernels" below.
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

// ---------------------------------------------------------------------------
// Device tables of the HIP kernels.  Per slot, the column-delta table holds a
// 64-bit entry: the delta (low word; 0 for the escape symbol) and the
// metadata (b - 1) | d << 16 | escape << 31; the value table holds the
// value's bits and the metadata b | d << 16 | escape << 31 (b the slot's
// base, at most 256, d its digit; unused slots have b = 1, d = 0).  The two
// metadata words are laid out so that one packed 16-bit multiply-add turns a
// (delta, value) pair of symbols into its digit pair and base product.
constexpr uint32_t kMetaEscape = 1u << 31;

// (R, D) of one nonzero's two symbols, delta s (meta (b_s - 1) | d_s << 16)
// then value t (meta b_t | d_t << 16), as (lo, hi) 16-bit halves:
// lo = (b_s - 1) b_t + b_t = b_s b_t, hi = d_s b_t + d_t (the value's digit is
// the less significant one).  Exact when every base is at most 255 (both
// results are below 2^16); escape bits must be clear.
DTANS_HD uint32_t pair_rd_ref(uint32_t ms, uint32_t mt) {
    const uint32_t bs1 = ms & 0xffffu, ds = ms >> 16, bt = mt & 0xffffu, dt = mt >> 16;
    return ((bs1 * bt + bt) & 0xffffu) | (((ds * bt + dt) & 0xffffu) << 16);
}

// A group of two nonzeros (symbols 1-4 or 5-8 of a segment) from the (R, D)
// pairs A (first nonzero) and B: D = D_A R_B + D_B, R = R_A R_B.
DTANS_HD void group_pairs_ref(uint32_t A, uint32_t B, uint32_t &D, uint32_t &R) {
    D = (A >> 16) * (B & 0xffffu) + (B >> 16);
    R = (A & 0xffffu) * (B & 0xffffu);
}

// The same group for tables with a base of 256 (16-bit halves would wrap):
// metadata of symbols 1-4 in stream order (delta, value, delta, value), D as
// above and Rm1 = R - 1 modulo 2^32 (R is at most 2^32).
DTANS_HD void group_general(uint32_t m0, uint32_t m1, uint32_t m2, uint32_t m3, uint32_t &D,
                            uint32_t &Rm1) {
    const uint32_t b0 = (m0 & 0xffffu) + 1u, b1 = m1 & 0xffffu;
    const uint32_t b2 = (m2 & 0xffffu) + 1u, b3 = m3 & 0xffffu;
    const uint32_t d0 = (m0 >> 16) & 0xffu, d1 = (m1 >> 16) & 0xffu;
    const uint32_t d2 = (m2 >> 16) & 0xffu, d3 = (m3 >> 16) & 0xffu;
    D = ((d0 * b1 + d1) * b2 + d2) * b3 + d3;  // < R <= 2^32
    Rm1 = b0 * b1 * b2 * b3 - 1u;              // wraps exactly when R = 2^32
}

#if defined(__HIPCC__) || defined(__HIP__)
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u16x2 as_u16x2(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t as_u32(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }

// pair_rd_ref as one v_pk_mad_u16 (the value's base broadcast to both halves)
__device__ __forceinline__ uint32_t pair_rd(uint32_t ms, uint32_t mt) {
    const u16x2 a = as_u16x2(ms), b = as_u16x2(mt);
    return as_u32(a * b.xx + b);
}

// group_pairs_ref: (D_A, 1) formed by one v_perm, D by one 16-bit dot product,
// R by one 24-bit multiply of the low halves
__device__ __forceinline__ void group_pairs(uint32_t A, uint32_t B, uint32_t &D, uint32_t &R) {
    const uint32_t U = __builtin_amdgcn_perm(1u, A, 0x0c040302u);  // (D_A, 1)
    D = __builtin_amdgcn_udot2(as_u16x2(U), as_u16x2(B), 0u, false);
    R = __umul24(A & 0xffffu, B & 0xffffu);
    // R < 2^32 is used as a 32-bit factor of the 64-bit state products; the
    // empty asm keeps the compiler from widening it to a 48-bit product
    // (which would double the 64-bit multiplies of append_word)
    asm("" : "+v"(R));
}
#endif

// Append a digit group (D, R) of a direct table (R = product of bases < 2^32)
// to the state (d, r) and run the check: true when the word is extracted
// from the state.  The extracted word is written either way (the caller uses
// it only then), which saves a select.
DTANS_HD bool append_word(uint32_t &d, uint32_t &r, uint32_t D, uint32_t R, uint32_t &word) {
    const uint64_t r64 = (uint64_t)r * R;
    const uint64_t d64 = (uint64_t)d * R + D;
    const bool extract = (r64 >> 32) != 0;
    word = (uint32_t)d64;
    d = extract ? (uint32_t)(d64 >> 32) : (uint32_t)d64;
    r = extract ? (uint32_t)(r64 >> 32) : (uint32_t)r64;
    return extract;
}

}  // namespace dtans
