// HIP kernels for gfx950: SpMV / SpMM / transpose / decode fused with dtANS
// decoding of CSR-dtANS streams, the fix-up of rows split across lanes, the
// persistent multi-matrix launch and the plain-CSR baseline.
//
// Work mapping (Sec. II-B and IV-B of Schaetzle, Pegolotti, Pueschel, "Fast
// Entropy Decoding for Sparse MVM on GPUs", 2026, with 64-lane wavefronts):
// one wavefront decodes one encoded wave (64 lane streams) at a time.  Every
// lane holds the state of its own stream; the conditional and unconditional
// word loads of a step are coalesced by a 64-bit ballot and a lane prefix
// count (v_mbcnt), as the paper does with a warp ballot and two popcounts.
// Both coding tables live in LDS for the whole (persistent) workgroup.
//
// Workgroups are persistent (a few per CU); each wavefront takes a contiguous
// range of encoded waves, and workgroups are renumbered so that those running
// on the same XCD (dispatch is round-robin over the 8 XCDs) own neighbouring
// ranges, which keeps their x gathers in the same L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <utility>
#include <vector>

#include "dtans_core.hpp"
#include "kernels.hpp"

namespace dtans {
namespace {

// How a lane holds a row: all of it; its end (the head: the row started in an
// earlier lane); its start (the tail: it continues in later lanes); or, in
// the nonzero layout, only a middle piece (started earlier, continues later).
constexpr int kComplete = 0, kHead = 1, kTail = 2, kMid = 3;
constexpr int kNumXcd = 8;
constexpr int kRingWords = 1024;  // per-wavefront LDS ring of the ring kernels (4 KiB)

__device__ __forceinline__ uint32_t lane_prefix(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// A load from a wave-uniform address through the scalar unit (constant
// address space): the value lands in SGPRs.  Only for data no kernel of the
// library writes while it runs (the matrix's offsets).
template <typename T>
__device__ __forceinline__ T uniform_load(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}

// Pointers into global memory for the decoder's loads.  A pointer the kernel
// read from device memory (the per-matrix views of the multi-matrix launches)
// is generic to the compiler, which then reads through it with flat
// instructions: 64-bit addresses, and counted against the LDS wait counter
// too, so that every wait for a table lookup would also wait for the gathers
// and stream words in flight.  Loads through these pointers are global loads
// whatever the pointer's origin (every matrix and vector is a device
// allocation).
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;
template <typename T>
using gmut = __attribute__((address_space(1))) T *;
// (the declared alignment is what the addresses guarantee: a load declared
// more aligned than its address lets the compiler draw wrong conclusions)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));                // 16-byte aligned
typedef uint32_t u32x4_a8 __attribute__((ext_vector_type(4), aligned(8)));  // 16 bytes, 8-byte aligned
typedef uint64_t u64_a4 __attribute__((aligned(4)));                        // 8 bytes, 4-byte aligned

template <typename VT> struct Bits;
template <> struct Bits<double> { typedef uint64_t T; };
template <> struct Bits<float> { typedef uint32_t T; };

template <typename VT>
__device__ __forceinline__ VT load_value(const void *p, uint64_t i) {
    return ((const VT *)p)[i];
}

// Value-table entry (device memory and LDS): the value's bits, then the slot's
// metadata b | d << 16 | escape << 31 (see dtans_core.hpp).  12 bytes for
// double: a value read is then two dword reads and the metadata a third, at
// 12 * slot, instead of a second table at another stride.
template <typename VT> struct VEntry;
template <> struct VEntry<double> {
    uint32_t lo, hi, meta;
    __device__ __forceinline__ double value() const {
        return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
    }
};
template <> struct VEntry<float> {
    uint32_t bits, meta;
    __device__ __forceinline__ float value() const { return __builtin_bit_cast(float, bits); }
};

// Both coding tables in LDS, the value table first so that every read of
// either has a constant offset below 2^16 (FP64: 48 + 32 KiB, FP32: 32 + 32).
template <typename VT> struct Tables {
    VEntry<VT> tv[kSlots];
    uint64_t td[kSlots];
};
static_assert(sizeof(VEntry<double>) == 12 && sizeof(VEntry<float>) == 8, "value entry sizes");
static_assert(sizeof(Tables<double>) == kSlots * 20 && sizeof(Tables<float>) == kSlots * 16,
              "tables are two packed arrays");

// ------------------------------------------------------------------ sinks
// A sink consumes one lane's decoded nonzeros a segment at a time:
//   segment<MULTI>(col, v, nreal, g, rowk): nonzeros k < nreal with columns
//     col[k] and values v[k]; nonzero k is number g + k in row-major order and
//     lies in row rowk[k].  MULTI is false when a lane holds a single row.
//     Every sink issues all its loads for the segment before it uses any.
//   finish_row(row, kind): row layout: the lane has seen its last nonzero of
//     `row`, which it holds whole.
//   finish_lane(row, kind, live): nonzero layout, called by every lane of the
//     wavefront together at the end of an encoded wave; `row` holds the live
//     lane's last nonzeros, `kind` how the lane holds it (kComplete, kHead,
//     kTail or kMid).
//   col_scale(params): the decoder multiplies every column delta by it, so
//     that col[k] arrives as column * col_scale modulo 2^32 (e.g. the byte
//     offset of x[column], which saves a shift per gather).
// Rows that end in the middle of a lane are finished inside segment().  Rows
// without nonzeros are a lane of their own in the row layout (finish_row with
// no segment) and never visited in the nonzero layout.

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// y (k columns) = alpha * A x + beta * y.  UNIT: k = 1 with unit strides and
// n * sizeof(VT) <= 2^32.
// ACC: accumulator type.  double everywhere except FP32 SpMM with many
// columns in the nonzero-balanced layout, where a lane sums a bounded number
// of nonzeros (at most 1024; measured error ~1e-7 of |A||x| at 512) before
// its partial sums are combined in double.
// DEFER (KC <= 4): a segment's x values are loaded when it arrives and
// multiplied at the start of the next decoding step (or when the lane ends),
// so their latency overlaps one step.  1: lanes hold single rows; 2: lanes
// may cross rows, and the rows of the deferred nonzeros are kept with them.
template <typename VT, int KC, bool UNIT, typename ACC = double, int DEFER = 0>
struct SpmmSink {
    static constexpr bool kCoop = false;
    // paired x loads (see segment); the general-table decoder runs without them
    static constexpr bool kPairs = UNIT && KC == 1 && sizeof(VT) == 8;
    static constexpr bool kPairs32 = UNIT && KC == 1 && sizeof(VT) == 4;  // per-lane pairs
    static_assert(!DEFER || KC <= 4, "deferred products keep 4*KC x values in registers");
    static constexpr int kOcc = KC <= 2 ? 8 : 4;  // waves per SIMD to allow
    struct Params {
        const VT *X;
        uint32_t ldx;
        VT *Y;
        uint32_t ldy;
        double *partial;  // [lane][head/tail][KC]
        double alpha, beta;
        // x holds at least two values, so that a read of two adjacent values
        // starting at column 0 stays inside it (the FP64 short segments and
        // the FP32 per-lane pairs in segment); 0 turns those reads off
        uint32_t pair_x = 0;
    };
    const Params p;
    int64_t lane;
    int32_t cur, head_row;  // row being accumulated; the lane's head row or -1
    ACC acc[KC];
    VT pv[DEFER ? 4 : 1], px[DEFER ? 4 : 1][KC];  // deferred segment
    int32_t prow[DEFER == 2 ? 4 : 1];             // its rows (DEFER 2)
    int pn;                                       // its nonzeros (0: none)
    // cur starts at -1: a row is finished only after the sink has seen one of
    // its nonzeros
    __device__ SpmmSink(const Params &pp, int64_t l, int32_t first_row, bool first_is_head)
        : p(pp), lane(l), cur(-1), head_row(first_is_head ? first_row : -1), pn(0) {
#pragma unroll
        for (int c = 0; c < KC; ++c) acc[c] = (ACC)0;
    }
    // multiply the deferred segment (its x loads were issued a step ago)
    __device__ __forceinline__ void consume() {
        if constexpr (DEFER == 1) {
            if (!ballot(pn < 4)) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int c = 0; c < KC; ++c) acc[c] = fma((ACC)pv[k], (ACC)px[k][c], acc[c]);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int c = 0; c < KC; ++c) {
                        const ACC t = fma((ACC)pv[k], (ACC)px[k][c], acc[c]);
                        acc[c] = k < pn ? t : acc[c];
                    }
            }
            pn = 0;
        } else if constexpr (DEFER == 2) {
            // rows never decrease along a lane: prow[3] == cur means no row ends
            if (!ballot(pn < 4 || prow[3] != cur)) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int c = 0; c < KC; ++c) acc[c] = fma((ACC)pv[k], (ACC)px[k][c], acc[c]);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < pn) {
                        if (prow[k] != cur) {
                            if (cur >= 0) store(cur, cur == head_row ? kHead : kComplete);
                            cur = prow[k];
                        }
#pragma unroll
                        for (int c = 0; c < KC; ++c) acc[c] = fma((ACC)pv[k], (ACC)px[k][c], acc[c]);
                    }
            }
            pn = 0;
        }
    }
    // called once per decoding step before the step issues any loads
    __device__ __forceinline__ void pre_step() { consume(); }
    // UNIT: x spans at most 4 GiB, so columns arrive as 32-bit byte offsets
    // from the uniform base (the decoder scales the deltas; base in SGPRs)
    static __device__ __forceinline__ uint32_t col_scale(const Params &) {
        return UNIT ? (uint32_t)sizeof(VT) : 1u;
    }
    __device__ __forceinline__ gptr<VT> xrow(uint32_t col) const {
        return UNIT ? (gptr<VT>)((const char *)p.X + col) : (gptr<VT>)(p.X + (uint64_t)col * p.ldx);
    }
    __device__ __forceinline__ void store(int32_t row, int kind) {
        if (kind == kComplete) {
            const gmut<VT> y = (gmut<VT>)(UNIT ? p.Y + row : p.Y + (uint64_t)(uint32_t)row * p.ldy);
#pragma unroll
            for (int c = 0; c < KC; ++c)
                y[c] = (VT)(p.beta == 0.0 ? p.alpha * (double)acc[c]
                                          : p.alpha * (double)acc[c] + p.beta * (double)y[c]);
        } else {
            double *q = p.partial + (2 * lane + (kind == kTail ? 1 : 0)) * KC;
#pragma unroll
            for (int c = 0; c < KC; ++c) q[c] = (double)acc[c];
        }
#pragma unroll
        for (int c = 0; c < KC; ++c) acc[c] = (ACC)0;
    }
    template <bool MULTI, bool PAIRS = kPairs>
    __device__ __forceinline__ void segment(const uint32_t col[4], const VT v[4], int nreal,
                                            int64_t, const int32_t rowk[4]) {
        if constexpr (DEFER) {
            static_assert(MULTI == (DEFER == 2), "DEFER 1 is for single-row lanes, 2 for the others");
            {
                // every lane loads four x values (column 0 stands in for
                // nonzeros past the lane's end; their products are dropped)
                uint32_t cc[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) cc[k] = col[k];
                if (ballot(nreal < 4)) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) cc[k] = k < nreal ? col[k] : 0u;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int c = 0; c < KC; ++c) px[k][c] = xrow(cc[k])[c];
#pragma unroll
                for (int k = 0; k < 4; ++k) pv[k] = v[k];
                if constexpr (DEFER == 2) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) prow[k] = rowk[k];
                }
                pn = nreal;
                return;
            }
        }
        if (KC * sizeof(VT) <= 32) {  // all four rows of X in flight at once
            VT x[4][KC];
            // common case, taken by the whole wavefront or not at all (a
            // uniform branch): no lane has a tail or a row end here
            if (!ballot(!(nreal >= 4 && (!MULTI || rowk[3] == cur)))) {
                if constexpr (PAIRS) {
                    // FP64 vector: when nonzeros k and k+1 of every lane are
                    // adjacent columns (uniform tests), one 16-byte load gives
                    // both x values.  The address unit takes such a load of a
                    // wavefront in the cycles of one 8-byte load (stencil and
                    // banded rows have runs of adjacent columns).
#pragma unroll
                    for (int k = 0; k < 4; k += 2) {
                        if (!ballot(col[k + 1] != col[k] + 8u)) {
                            // (an offset the compiler cannot share with the
                            // other branch: a shared address would be formed
                            // as a 64-bit pointer ahead of the branch, where
                            // this form keeps the base in SGPRs)
                            uint32_t o = col[k];
                            asm("" : "+v"(o));
                            const u32x4_a8 q = *(gptr<u32x4_a8>)((const char *)p.X + o);
                            x[k][0] = __builtin_bit_cast(VT, (uint64_t)q.y << 32 | q.x);
                            x[k + 1][0] = __builtin_bit_cast(VT, (uint64_t)q.w << 32 | q.z);
                        } else {
                            x[k][0] = xrow(col[k])[0];
                            x[k + 1][0] = xrow(col[k + 1])[0];
                        }
                    }
                } else if constexpr (kPairs32) {
                    // FP32 vector, pairs per lane: an 8-byte load ending at
                    // column k+1 gives x at k+1 and, in the lanes whose
                    // columns k and k+1 are adjacent, x at k too; only the
                    // other lanes load x at k on their own, so the address
                    // unit sees their cache lines only (half the lanes of a
                    // weight pruned to half its entries).  The load starts at
                    // column 0 when column k+1 is 0 (repeated columns), so it
                    // stays inside x once x holds two values.
                    // (every load is issued before any value is selected,
                    // so that no wait comes between them)
                    if (p.pair_x) {  // uniform
                        uint64_t q[2];
                        VT xs[2];
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const uint32_t c1 = col[2 * h + 1];
                            q[h] = *(gptr<u64_a4>)((const char *)p.X + (c1 >= 4u ? c1 - 4u : 0u));
                        }
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            xs[h] = (VT)0;
                            if (col[2 * h] + 4u != col[2 * h + 1]) xs[h] = xrow(col[2 * h])[0];
                        }
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const uint32_t c1 = col[2 * h + 1];
                            const VT lo = __builtin_bit_cast(VT, (uint32_t)q[h]);
                            const VT hi = __builtin_bit_cast(VT, (uint32_t)(q[h] >> 32));
                            x[2 * h + 1][0] = c1 >= 4u ? hi : lo;
                            x[2 * h][0] = col[2 * h] + 4u == c1 ? lo : xs[h];
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < 4; ++k) x[k][0] = xrow(col[k])[0];
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
#pragma unroll
                        for (int c = 0; c < KC; ++c) x[k][c] = xrow(col[k])[c];
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int c = 0; c < KC; ++c) acc[c] = fma((ACC)v[k], (ACC)x[k][c], acc[c]);
                return;
            }
            if constexpr (!MULTI) {
                // single-row lanes: only a lane's last segment is short (or it
                // has none left); column 0 stands in for the missing nonzeros,
                // whose products are dropped by a select, with no branches
                if constexpr (PAIRS) {
                    // Pairs as in the common case when both pairs of every
                    // lane holding them are adjacent (a uniform test) and x
                    // holds at least two values.  A lane holding both
                    // nonzeros of a pair reads them at the first column; a
                    // lane holding only the first reads the 16 bytes that end
                    // at its column (or start at column 0), a lane holding
                    // neither reads columns 0 and 1: every read stays inside
                    // x.
                    if (p.pair_x && !ballot((1 < nreal && col[1] != col[0] + 8u) ||
                                            (3 < nreal && col[3] != col[2] + 8u))) {
                        bool up[2];
                        u32x4_a8 q[2];
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int k = 2 * h;
                            const bool one = k < nreal, both = k + 1 < nreal;
                            up[h] = one && !both && col[k] != 0u;
                            const uint32_t off = both ? col[k] : (up[h] ? col[k] - 8u : 0u);
                            q[h] = *(gptr<u32x4_a8>)((const char *)p.X + off);
                        }
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const VT lo = __builtin_bit_cast(VT, (uint64_t)q[h].y << 32 | q[h].x);
                            const VT hi = __builtin_bit_cast(VT, (uint64_t)q[h].w << 32 | q[h].z);
                            x[2 * h][0] = up[h] ? hi : lo;
                            x[2 * h + 1][0] = hi;
                        }
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const ACC t = fma((ACC)v[k], (ACC)x[k][0], acc[0]);
                            acc[0] = k < nreal ? t : acc[0];
                        }
                        return;
                    }
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t cc = k < nreal ? col[k] : 0u;
#pragma unroll
                    for (int c = 0; c < KC; ++c) x[k][c] = xrow(cc)[c];
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int c = 0; c < KC; ++c) {
                        const ACC t = fma((ACC)v[k], (ACC)x[k][c], acc[c]);
                        acc[c] = k < nreal ? t : acc[c];
                    }
                return;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < nreal)
#pragma unroll
                    for (int c = 0; c < KC; ++c) x[k][c] = xrow(col[k])[c];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k < nreal) {
                    if (MULTI && rowk[k] != cur) {
                        if (cur >= 0) store(cur, cur == head_row ? kHead : kComplete);
                        cur = rowk[k];
                    }
#pragma unroll
                    for (int c = 0; c < KC; ++c) acc[c] = fma((ACC)v[k], (ACC)x[k][c], acc[c]);
                }
        } else {
            // wider rows of X: load nonzero k+1 while multiplying nonzero k
            VT xa[KC], xb[KC];
            if (nreal > 0) {
#pragma unroll
                for (int c = 0; c < KC; ++c) xa[c] = xrow(col[0])[c];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                VT *xc = (k & 1) ? xb : xa;
                VT *xn = (k & 1) ? xa : xb;
                if (k + 1 < 4 && k + 1 < nreal) {
#pragma unroll
                    for (int c = 0; c < KC; ++c) xn[c] = xrow(col[k + 1])[c];
                }
                if (k < nreal) {
                    if (MULTI && rowk[k] != cur) {
                        if (cur >= 0) store(cur, cur == head_row ? kHead : kComplete);
                        cur = rowk[k];
                    }
#pragma unroll
                    for (int c = 0; c < KC; ++c) acc[c] = fma((ACC)v[k], (ACC)xc[c], acc[c]);
                }
            }
        }
    }
    __device__ __forceinline__ void finish_row(int32_t row, int kind) {
        consume();
        store(row, kind);
    }
    // Middle pieces of a row are summed across the wavefront first: a
    // segmented suffix sum over consecutive lanes holding middles of the same
    // row (rows never decrease along the lanes, so equal rows d lanes apart
    // mean the whole stretch holds that row), after which only the first
    // such lane of each stretch stores (its head slot).  The fix-up then reads
    // one partial per wavefront a row spans instead of one per lane.
    __device__ __forceinline__ void finish_lane(int32_t row, int kind, bool live) {
        consume();
        const uint32_t wl = (uint32_t)lane & (kWave - 1);
        const bool mid = live && kind == kMid;
        const int32_t key = mid ? row : -1;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int32_t kd = __shfl_down(key, d);
            const bool ok = mid && wl + d < (uint32_t)kWave && kd == key;
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                const ACC t = __shfl_down(acc[c], d);
                if (ok) acc[c] += t;
            }
        }
        const int32_t kp = __shfl_up(key, 1);
        if (mid) {
            if (wl == 0 || kp != key) store(row, kHead);
        } else if (live) {
            store(row, kind);
        }
    }
};

// A 32-bit value of lane `src` (all lanes of the wavefront active)
__device__ __forceinline__ uint32_t lane_value(uint32_t v, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)v);
}
template <typename T>
__device__ __forceinline__ T lane_value_of(T v, uint32_t src) {
    if constexpr (sizeof(T) == 8) {
        const uint64_t b = __builtin_bit_cast(uint64_t, v);
        const uint64_t r = (uint64_t)lane_value((uint32_t)b, src) |
                           ((uint64_t)lane_value((uint32_t)(b >> 32), src) << 32);
        return __builtin_bit_cast(T, r);
    } else {
        return __builtin_bit_cast(T, lane_value(__builtin_bit_cast(uint32_t, v), src));
    }
}

// Y (KC = G * CL columns) = alpha * A X + beta * Y with G lanes per row of X.
// The 64 lanes of a wavefront form 64 / G groups; group q keeps, in G slots,
// the sums of the streams q*G .. q*G + G - 1 (slot i: stream q*G + i), each
// lane for CL = 16 / sizeof(VT) consecutive columns (one 16-byte load per
// nonzero).  A step's (column, value) pairs move from the decoding lane to
// its group with ds_bpermute, so that one load instruction reads 64 / G whole
// rows of X (the address unit takes one cache line of an instruction at a
// time: rows read one per lane cost a line per lane).  Columns arrive as byte
// offsets of rows of X (col_scale = ldx * sizeof(VT)); X and Y rows are
// 16-byte aligned.  Rows split over lanes give the same partial sums as
// SpmmSink (tail and head slots; the middle pieces of a row summed per
// wavefront into the head slot of the stretch's first stream), so the same
// fix-up finishes them.
template <typename VT, int G, typename ACC = double>
struct CoopSpmmSink {
    static constexpr bool kCoop = true;
    static constexpr bool kPairs = false;
    static constexpr int CL = 16 / (int)sizeof(VT), KC = G * CL, NG = kWave / G;
    // waves per SIMD to allow: with eight slots per lane the accumulators and
    // the rows of X in flight do not fit beside the decoder in 128 registers;
    // with two or four, 168 registers avoid spills (measured faster than four
    // waves per SIMD with spills, and than two)
    static constexpr int kOcc = G >= 8 ? 2 : 3;
    static_assert(G == 2 || G == 4 || G == 8, "2, 4 or 8 lanes per row of X");
    struct Params {
        const VT *X;
        uint32_t ldx;
        VT *Y;
        uint32_t ldy;
        double *partial;  // [lane][head/tail][KC]
        double alpha, beta;
    };
    const Params p;
    uint32_t grp, part;      // group, column chunk of this lane
    int64_t wave0;           // global index of stream 0 of the wave
    ACC acc[G][CL];
    int32_t cur[G];          // row being summed in slot i (-1 before the first nonzero)
    int32_t head_row[G];     // the slot's first row when it began before the stream, else -1
    int32_t last;            // row of this lane's last nonzero so far (-1 before the first)

    static __device__ __forceinline__ uint32_t col_scale(const Params &pp) {
        return pp.ldx * (uint32_t)sizeof(VT);
    }
    __device__ CoopSpmmSink(const Params &pp, int64_t l, int32_t first_row, bool first_is_head) : p(pp) {
        const uint32_t lane = (uint32_t)l & (kWave - 1);
        grp = lane / G;
        part = lane % G;
        wave0 = l - lane;
        last = -1;
        const int32_t hr = first_is_head ? first_row : -1;
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const uint32_t src = grp * G + i;
            cur[i] = -1;
            head_row[i] = (int32_t)lane_value((uint32_t)hr, src);
#pragma unroll
            for (int c = 0; c < CL; ++c) acc[i][c] = (ACC)0;
        }
    }
    __device__ __forceinline__ void pre_step() {}
    __device__ __forceinline__ VT *yrow(int32_t row) const {
        return p.Y + (uint64_t)(uint32_t)row * p.ldy + part * CL;
    }
    __device__ __forceinline__ double *slot(int64_t stream, int kind) const {
        return p.partial + (2 * stream + (kind == kTail ? 1 : 0)) * KC + part * CL;
    }
    // store slot i's sums for `row` (kind as for SpmmSink::store) and clear them
    __device__ __forceinline__ void store(int i, int32_t row, int kind) {
        if (kind == kComplete) {
            VT *y = yrow(row);
#pragma unroll
            for (int c = 0; c < CL; ++c)
                y[c] = (VT)(p.beta == 0.0 ? p.alpha * (double)acc[i][c]
                                          : p.alpha * (double)acc[i][c] + p.beta * (double)y[c]);
        } else {
            double *q = slot(wave0 + grp * G + i, kind);
#pragma unroll
            for (int c = 0; c < CL; ++c) q[c] = (double)acc[i][c];
        }
#pragma unroll
        for (int c = 0; c < CL; ++c) acc[i][c] = (ACC)0;
    }
    template <bool MULTI>
    __device__ __forceinline__ void segment(const uint32_t col[4], const VT v[4], int nreal, int64_t,
                                            const int32_t rowk[4]) {
        // some stream reaches a row it did not end the last step in (a
        // uniform test); otherwise the slots' rows stay as they are
        const bool moved = MULTI && ballot(nreal > 0 && rowk[nreal - 1] != last) != 0;
        if (MULTI && nreal > 0) last = rowk[nreal - 1];
        int nr[G];
#pragma unroll
        for (int i = 0; i < G; ++i) nr[i] = (int)lane_value((uint32_t)nreal, grp * G + i);
        // rounds r = 4 i + j (nonzero j of slot i's stream), each row of X
        // requested kAhead rounds before it is multiplied
        constexpr int R = 4 * G, kAhead = 2;
        uint4 xs[kAhead];
        VT vv[kAhead];
        int32_t rk[kAhead];
        auto fetch = [&](int r) {
            const int b = r % kAhead, i = r >> 2, j = r & 3;
            const uint32_t src = grp * G + i;
            const uint32_t cj = lane_value(col[j], src);
            vv[b] = lane_value_of(v[j], src);
            if (MULTI && moved) rk[b] = (int32_t)lane_value((uint32_t)rowk[j], src);
            // nonzeros past a stream's end read row 0 of X (their products are dropped)
            xs[b] = *(const uint4 *)((const char *)p.X + (j < nr[i] ? cj : 0u) + part * 16);
        };
#pragma unroll
        for (int r = 0; r < kAhead && r < R; ++r) fetch(r);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int b = r % kAhead, i = r >> 2, j = r & 3;
            VT x[CL];
            __builtin_memcpy(x, &xs[b], 16);
            const VT vr = vv[b];
            const int32_t rr = (MULTI && moved) ? rk[b] : 0;
            if (r + kAhead < R) fetch(r + kAhead);
            if (j < nr[i]) {
                if (MULTI && moved && rr != cur[i]) {
                    if (cur[i] >= 0) store(i, cur[i], cur[i] == head_row[i] ? kHead : kComplete);
                    cur[i] = rr;
                }
#pragma unroll
                for (int c = 0; c < CL; ++c) acc[i][c] = fma((ACC)vr, (ACC)x[c], acc[i][c]);
            }
        }
    }
    // single-row streams (row layout): every lane calls this at the end of the
    // wave; `live` lanes' rows are complete
    __device__ __forceinline__ void finish_row(int32_t row, int kind) { finish_all(row, kind, true); }
    __device__ __forceinline__ void finish_lane(int32_t row, int kind, bool live) { finish_all(row, kind, live); }

    __device__ __forceinline__ void finish_all(int32_t row, int kind, bool live) {
        int32_t rw[G], key[G];
        int kd[G];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const uint32_t src = grp * G + i;
            rw[i] = (int32_t)lane_value((uint32_t)row, src);
            kd[i] = (int)lane_value((uint32_t)(live ? kind : -1), src);
            key[i] = kd[i] == kMid ? rw[i] : -1;
        }
        // non-middle pieces: complete rows to Y, heads and tails to their slots
#pragma unroll
        for (int i = 0; i < G; ++i)
            if (kd[i] >= 0 && kd[i] != kMid) store(i, rw[i], kd[i]);
        // middle pieces: suffix sums over the wave's streams in order (slots
        // of a group, then groups), keyed by row (rows never decrease along
        // the streams, so equal keys far apart mean the whole stretch holds
        // that row); the first stream of each stretch stores the total
#pragma unroll
        for (int i = G - 2; i >= 0; --i)
            if (key[i] >= 0 && key[i + 1] == key[i]) {
#pragma unroll
                for (int c = 0; c < CL; ++c) acc[i][c] += acc[i + 1][c];
            }
        const int32_t k0 = key[0];
        const int32_t kn = (int32_t)lane_value((uint32_t)k0, ((grp + 1) % NG) * G + part);
        const int32_t kprev = (int32_t)lane_value((uint32_t)key[G - 1], ((grp + NG - 1) % NG) * G + part);
        bool kok[6];  // the cross-group steps that join equal keys
#pragma unroll
        for (int t = 0, d = 1; d < NG; d <<= 1, ++t) {
            const int32_t kdn = (int32_t)lane_value((uint32_t)k0, ((grp + d) % NG) * G + part);
            kok[t] = k0 >= 0 && grp + d < (uint32_t)NG && kdn == k0;
        }
#pragma unroll
        for (int c = 0; c < CL; ++c) {
            ACC V = acc[0][c];
#pragma unroll
            for (int t = 0, d = 1; d < NG; d <<= 1, ++t) {
                const ACC u = lane_value_of(V, ((grp + d) % NG) * G + part);
                if (kok[t]) V += u;
            }
            // the next group's slot-0 total
            const ACC Vn = lane_value_of(V, ((grp + 1) % NG) * G + part);
#pragma unroll
            for (int i = 0; i < G; ++i) {
                if (key[i] < 0) continue;
                const bool first = i > 0 ? key[i - 1] != key[i] : (grp == 0 || kprev != key[i]);
                if (!first) continue;
                const bool more = key[G - 1] == key[i] && grp + 1 < (uint32_t)NG && kn == key[i];
                const ACC tot = i == 0 ? V : acc[i][c] + (more ? Vn : (ACC)0);
                slot(wave0 + grp * G + i, kHead)[c] = (double)tot;
            }
        }
    }
};

// dX (k columns) += alpha * A^T dY, scattered with atomic adds.
template <typename VT, int KC>
struct TransSink {
    static constexpr bool kCoop = false;
    static constexpr bool kPairs = false;
    static constexpr int kOcc = KC <= 2 ? 8 : 4;
    struct Params {
        const VT *dY;
        uint32_t lddy;
        VT *dX;
        uint32_t lddx;
        double alpha;
    };
    const Params p;
    int32_t cur;
    VT dy[KC];
    static __device__ __forceinline__ uint32_t col_scale(const Params &) { return 1u; }
    __device__ TransSink(const Params &pp, int64_t, int32_t first_row, bool) : p(pp), cur(-1) {
        (void)first_row;
    }
    __device__ __forceinline__ void load_row(int32_t row) {
        cur = row;
        const VT *src = p.dY + (uint64_t)(uint32_t)row * p.lddy;
#pragma unroll
        for (int c = 0; c < KC; ++c) dy[c] = (VT)(p.alpha * (double)src[c]);
    }
    template <bool MULTI>
    __device__ __forceinline__ void segment(const uint32_t col[4], const VT v[4], int nreal,
                                            int64_t, const int32_t rowk[4]) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nreal) {
                if (rowk[k] != cur) load_row(rowk[k]);
                VT *dst = p.dX + (uint64_t)col[k] * p.lddx;
#pragma unroll
                for (int c = 0; c < KC; ++c) unsafeAtomicAdd(dst + c, v[k] * dy[c]);
            }
    }
    __device__ __forceinline__ void pre_step() {}
    __device__ __forceinline__ void finish_row(int32_t, int) {}
    __device__ __forceinline__ void finish_lane(int32_t, int, bool) {}
};

// Position of element i of the LDS block of dX: one spare slot after every 32,
// so that lanes whose columns lie a multiple of 32 / KC apart (equal lane
// lengths over a regular row walk exactly such strides) do not all hit one
// LDS bank.
__device__ __forceinline__ uint32_t lds_slot(uint32_t i) { return i + (i >> 5); }

// dX (k columns) += A^T dY into a block of dX in LDS (trans_lds_kernel);
// alpha is applied when the copies are summed
template <typename VT, int KC>
struct TransLdsSink {
    static constexpr bool kCoop = false;
    static constexpr bool kPairs = false;
    static constexpr int kOcc = 4;
    struct Params {
        const VT *dY;
        uint32_t lddy;
        VT *lds;  // n x KC, set by the kernel
    };
    const Params p;
    int32_t cur;
    VT dy[KC];
    static __device__ __forceinline__ uint32_t col_scale(const Params &) { return 1u; }
    __device__ TransLdsSink(const Params &pp, int64_t, int32_t, bool) : p(pp), cur(-1) {}
    __device__ __forceinline__ void load_row(int32_t row) {
        cur = row;
        const VT *src = p.dY + (uint64_t)(uint32_t)row * p.lddy;
#pragma unroll
        for (int c = 0; c < KC; ++c) dy[c] = src[c];
    }
    template <bool MULTI>
    __device__ __forceinline__ void segment(const uint32_t col[4], const VT v[4], int nreal,
                                            int64_t, const int32_t rowk[4]) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nreal) {
                if (rowk[k] != cur) load_row(rowk[k]);
#pragma unroll
                for (int c = 0; c < KC; ++c) atomicAdd(p.lds + lds_slot(col[k] * KC + c), v[k] * dy[c]);
            }
    }
    __device__ __forceinline__ void pre_step() {}
    __device__ __forceinline__ void finish_row(int32_t, int) {}
    __device__ __forceinline__ void finish_lane(int32_t, int, bool) {}
};

// decode to CSR: column and value bits of every nonzero
template <typename VT>
struct DecodeSink {
    static constexpr bool kCoop = false;
    static constexpr bool kPairs = false;
    static constexpr int kOcc = 8;
    struct Params {
        int32_t *col;
        typename Bits<VT>::T *vals;
    };
    const Params p;
    static __device__ __forceinline__ uint32_t col_scale(const Params &) { return 1u; }
    __device__ DecodeSink(const Params &pp, int64_t, int32_t, bool) : p(pp) {}
    template <bool MULTI>
    __device__ __forceinline__ void segment(const uint32_t col[4], const VT v[4], int nreal,
                                            int64_t g, const int32_t *) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nreal) {
                p.col[g + k] = (int32_t)col[k];
                p.vals[g + k] = __builtin_bit_cast(typename Bits<VT>::T, v[k]);
            }
    }
    __device__ __forceinline__ void pre_step() {}
    __device__ __forceinline__ void finish_row(int32_t, int) {}
    __device__ __forceinline__ void finish_lane(int32_t, int, bool) {}
};

// --------------------------------------------------------- wave decoding
// Word sources.  A decoder reads the words of its wave's stream at 32-bit
// byte offsets that are wave-uniform plus a lane prefix.
//
// GlobalWords reads them from device memory: every step's loads depend on the
// previous step's ballots, so each step waits for one memory round trip.
struct GlobalWords {
    const char *W;   // stream base of the current encoded wave
    // its length, kept in 64 bits: a narrower copy would leave half of the
    // loaded offset unused, and reusing that register before the load has
    // returned makes the wave wait for it
    uint64_t bytes;
    // the word at byte offset pos (uniform) + 4 * (lanes of mask below this one):
    // the base stays fixed in SGPRs and each lane forms its 32-bit offset with
    // one shift-add (readfirstlane keeps pos a scalar sum, which the compiler
    // would otherwise fold into the lane count)
    __device__ __forceinline__ uint32_t read(uint32_t pos, uint64_t mask) const {
        const uint32_t p = __builtin_amdgcn_readfirstlane(pos);
        return *(gptr<uint32_t>)(W + (p + 4 * lane_prefix(mask)));
    }
    // the same when every lane of the wavefront reads (prefix = lane)
    __device__ __forceinline__ uint32_t read_lanes(uint32_t pos, uint32_t lane) const {
        const uint32_t p = __builtin_amdgcn_readfirstlane(pos);
        return *(gptr<uint32_t>)(W + (p + 4 * lane));
    }
    // the word at byte offset pos (uniform) + off (per lane): escapes stored
    // in the stream
    __device__ __forceinline__ uint32_t word_at(uint32_t pos, uint32_t off) const {
        const uint32_t p = __builtin_amdgcn_readfirstlane(pos);
        return *(gptr<uint32_t>)(W + (p + off));
    }
    // Nothing in the memory system fetches a stream ahead of its reads, so
    // every step's words would come from HBM.  Once the first words are
    // requested, one load per lane touches the next 64 cache lines (128 B)
    // of the stream, which brings them into L2 while the first steps run.
    // The value is kept (retire) so that the load is not removed; loads
    // complete in order, so the steps' own waits already cover it.
    __device__ __forceinline__ uint32_t prefetch(uint32_t pos, uint32_t lane) const {
        const uint32_t o = (pos & ~127u) + 128u * (lane + 1);
        return o < bytes ? *(gptr<uint32_t>)(W + o) : 0u;
    }
    __device__ __forceinline__ void retire(uint32_t v) const { asm volatile("" ::"v"(v)); }
    __device__ __forceinline__ void step_begin() {}
    __device__ __forceinline__ void consumed(uint32_t) {}
};

// RingWords stages a contiguous run of streams (the encoded waves [a, b) of
// one wavefront are adjacent in memory) through a per-wavefront ring of kRing
// words in LDS.  Chunks of 1 KiB (one aligned 16-byte load per lane) are requested
// as soon as the ring has room and written into it at the start of the next
// step, so the words a step reads were loaded at least one step earlier and
// the decode's serial chain runs through LDS only.  Invariant: chunks are
// requested in order, at most one per step, and written one step later,
// after that step's reads; a step reads at most 768 bytes (three words per
// lane) < one chunk, so the requested end stays at least kRing*4 - 1 KiB
// ahead of the read position, and the words a step reads were requested two
// steps earlier: kRing*4 - 1 KiB >= 2 * 768 + 768 bytes suffices.  A chunk
// overwrites only words already read.  LDS operations of one wavefront
// complete in order, so no barrier is needed between chunk writes and reads.
template <int kRing>
struct RingWords {
    static constexpr uint32_t kChunk = 1024;
    // the first kMirror words of the ring are kept a second time after its
    // end, so that the at most 64 words one read instruction spans never
    // wrap: a read is a prefix count from a uniform start, as from memory
    static constexpr int kMirror = 64;
    static constexpr int kWords = kRing + kMirror;  // LDS words per wavefront
    static_assert(kRing * 4 >= (int)kChunk + 3 * 768, "ring too small for two steps of lead");
    static_assert((kRing & (kRing - 1)) == 0 && kRing % 256 == 0, "ring of whole chunks");
    uint32_t *ring;     // this wavefront's ring (kWords words)
    const char *base;   // the run's first word rounded down to 16 bytes
    uint32_t skew;      // bytes from base to the run's first word (0..12)
    uint32_t total;     // skew + bytes in the run
    uint32_t fetched;   // bytes from base requested so far (multiple of kChunk)
    uint32_t pend_at;   // offset from base of the chunk in flight
    bool has_pend;
    uint4 pend;         // this lane's 16 bytes of the chunk in flight
    uint32_t lane;

    // 16-byte aligned loads; the last one of a run passes its end by at most
    // 15 bytes, which stay inside the padded word buffer.  Lanes past the end
    // reload the run's first 16 bytes (unconditional loads keep the wait
    // counts static); what they write to the ring is never read.
    __device__ __forceinline__ uint4 load_chunk_part(uint32_t at) const {
        const uint32_t o = at + 16 * lane;
        return *(const uint4 *)(base + (o < total ? o : 0u));
    }
    __device__ __forceinline__ void write_chunk_part(uint32_t at, uint4 v) {
        const uint32_t i = ((at >> 2) + 4 * lane) & (kRing - 1);
        *(uint4 *)(ring + i) = v;
        if (i < kMirror) *(uint4 *)(ring + kRing + i) = v;
    }
    __device__ __forceinline__ void start(uint32_t *r, const uint32_t *first, uint32_t bytes,
                                          uint32_t ln) {
        ring = r;
        skew = (uint32_t)((uintptr_t)first & 15);
        base = (const char *)first - skew;
        total = skew + bytes;
        lane = ln;
        fetched = 0;
        has_pend = false;
        // fill the whole ring before the first read
#pragma unroll
        for (int c = 0; c < kRing * 4 / (int)kChunk; ++c) {
            if (fetched < total) {
                write_chunk_part(fetched, load_chunk_part(fetched));
                fetched += kChunk;
            }
        }
    }
    // pos: bytes from the run's first word (uniform, so the start address is
    // scalar work); the lane adds its prefix count
    __device__ __forceinline__ uint32_t read(uint32_t pos, uint64_t mask) const {
        const uint32_t *at = ring + (((pos + skew) >> 2) & (kRing - 1));
        return at[lane_prefix(mask)];
    }
    __device__ __forceinline__ uint32_t read_lanes(uint32_t pos, uint32_t ln) const {
        const uint32_t *at = ring + (((pos + skew) >> 2) & (kRing - 1));
        return at[ln];
    }
    // from memory (streams with escapes inside are never staged through a
    // ring: a step may read more of them than the ring holds ahead)
    __device__ __forceinline__ uint32_t word_at(uint32_t pos, uint32_t off) const {
        const uint32_t p = __builtin_amdgcn_readfirstlane(pos);
        return *(const uint32_t *)(base + (p + skew + off));
    }
    __device__ __forceinline__ uint32_t prefetch(uint32_t, uint32_t) const { return 0u; }
    __device__ __forceinline__ void retire(uint32_t) const {}
    __device__ __forceinline__ void step_begin() {
        if (has_pend) {
            write_chunk_part(pend_at, pend);
            has_pend = false;
        }
    }
    // the decoder's read position has advanced to pos (bytes from the run's
    // first word); request the next chunk once the ring has room for it
    __device__ __forceinline__ void consumed(uint32_t pos) {
        if (fetched < total && fetched + kChunk <= pos + skew + kRing * 4) {
            pend = load_chunk_part(fetched);
            pend_at = fetched;
            has_pend = true;
            fetched += kChunk;
        }
    }
};

// Read positions of a stream: words (bytes), escaped deltas and escaped values
// (counts), with the escape region bases.  A cursor restarts at every encoded
// wave for GlobalWords and runs on across a run for RingWords.
template <typename VT>
struct Cursor {
    uint32_t pos, dpos, vpos;
    const uint32_t *ED;
    const VT *EV;
};

// Where a lane's stream sits in the matrix: its first nonzero g0 and count
// (the row layout keeps only the row's [beg, end)); the row of that nonzero
// with the row's [beg, end).  The nonzero layout
// walks the list of nonempty rows ({row, end} pairs, a sentinel {m, nnz} at
// the end), so a lane never visits empty rows (their y is written by
// empty_rows_kernel) and crosses exactly one row per nonzero that starts one;
// it keeps the next two list entries loaded ahead (n1, n2).  Finding the
// first entry takes two dependent loads (lane_row, then the list), so
// callers may issue the first a wave ahead (lane_first_row).
struct LaneGeo {
    int64_t g0;
    int cnt;
    int32_t krow;  // layout NNZ: index of `row` in the nonempty-row list
    int32_t row, row_beg, row_end;
    int2 n1, n2;
    // layout ROW: the row of the original matrix this lane's row is (rows
    // sorted within windows are encoded in that order) and the position of
    // its first nonzero there
    int32_t orow;
    int64_t gout;
};

template <int LAYOUT>
__device__ __forceinline__ int32_t lane_first_row(const DevMat &a, int64_t slice, uint32_t lane) {
    const int64_t l = slice * kWave + lane;
    if (l >= a.num_lanes) return 0;
    return LAYOUT == 1 ? (int32_t)l : a.lane_row[l];
}

template <int LAYOUT>
__device__ __forceinline__ LaneGeo lane_geo(const DevMat &a, int64_t slice, uint32_t lane,
                                            int32_t first) {
    LaneGeo q{0, 0, 0, 0, 0, 0, make_int2(0, 0), make_int2(0, 0), 0, 0};
    const int64_t l = slice * kWave + lane;
    if constexpr (LAYOUT == 1) {
        // the row's bounds only (lanes past the last row read the last
        // row's): the count is formed where the wave starts, so that a wave
        // loading the next one's geometry does not wait for it
        const int64_t lc = l < a.num_lanes ? l : a.num_lanes - 1;
        q.row = first;
        q.row_beg = ((gptr<int32_t>)a.row_ptr)[lc];
        q.row_end = ((gptr<int32_t>)a.row_ptr)[lc + 1];
        q.orow = first;
        q.gout = q.row_beg;
        if (a.row_perm) {  // uniform
            q.orow = ((gptr<int32_t>)a.row_perm)[lc];
            q.gout = ((gptr<int32_t>)a.orig_row_ptr)[q.orow];
        }
    } else if (l < a.num_lanes) {
        q.g0 = l * (int64_t)a.lane_nnz;
        q.cnt = (int)min((int64_t)a.lane_nnz, a.nnz - q.g0);
        q.krow = first;
        const int2 c = a.nzr[first];
        q.row = c.x;
        q.row_end = c.y;
        q.row_beg = first > 0 ? a.nzr[first - 1].y : 0;
        q.n1 = a.nzr[min((int64_t)first + 1, a.n_nzr)];
        q.n2 = a.nzr[min((int64_t)first + 2, a.n_nzr)];
    }
    return q;
}

// LDS byte offsets of a segment's eight slots (unpack8 of dtans_core.hpp
// with the entry sizes folded in): delta slots i1, i3, i5, i7 into the delta
// table (8-byte entries), value slots i2, i4, i6, i8 into the value table
// (E-byte entries), straight from the three words.
template <int E>
__device__ __forceinline__ void slot_offsets(uint32_t w1, uint32_t w2, uint32_t w3, uint32_t od[4],
                                             uint32_t ov[4]) {
    od[0] = (w3 << 3) & 0x7ff8u;                                  // i1 = w3[0:12]
    ov[0] = ((w3 >> 12) & 0xfffu) * E;                             // i2 = w3[12:24]
    od[1] = __builtin_amdgcn_alignbit(w2, w3, 21) & 0x7ff8u;       // i3 = w3[24:32] | w2[0:4] << 8
    ov[1] = ((w2 >> 4) & 0xfffu) * E;                              // i4 = w2[4:16]
    od[2] = (w2 >> 13) & 0x7ff8u;                                  // i5 = w2[16:28]
    ov[2] = (__builtin_amdgcn_alignbit(w1, w2, 28) & 0xfffu) * E;  // i6 = w2[28:32] | w1[0:8] << 4
    od[3] = (w1 >> 5) & 0x7ff8u;                                   // i7 = w1[8:20]
    ov[3] = (w1 >> 20) * E;                                        // i8 = w1[20:32]
}

// Decode encoded wave `slice` (lanes slice*64 .. slice*64+63) and feed the
// nonzeros of this thread's lane to a sink constructed here.
// TF, the table format: 0 some base is 256 (the paper's M; a digit group's
// base product may reach 2^32); 1 "direct" tables (every base at most 255: a
// group's arithmetic runs on packed 16-bit halves); 2 direct tables without
// an escape symbol in either alphabet (no escape checks at all).
// A step of the whole wavefront is "full" when every lane decodes four
// nonzeros and has a next segment (no masks, every lane loads its words);
// other steps handle lanes that end, are short or have nothing left.
template <int LAYOUT, typename VT, class Sink, class Src, int TF>
__device__ __forceinline__ void decode_slice(const DevMat &a, const Tables<VT> &tb, int64_t slice,
                                             uint32_t lane, const typename Sink::Params &sp,
                                             Src &src, Cursor<VT> &cur, const LaneGeo &geo) {
    const int64_t l = slice * kWave + lane;
    const bool live = l < a.num_lanes;
    const int64_t g0 = LAYOUT == 1 ? (int64_t)geo.row_beg : geo.g0;
    const int cnt = LAYOUT == 1 ? (live ? geo.row_end - geo.row_beg : 0) : geo.cnt;
    int32_t row = geo.row, row_beg = geo.row_beg, row_end = geo.row_end, krow = geo.krow;
    int2 n1 = geo.n1, n2 = geo.n2;
    // the sink sees rows and nonzero positions of the original matrix (row
    // layout: rows may be encoded in another order); the decoder's own row
    // (first deltas) is the encoded one
    const int32_t srow = LAYOUT == 1 ? geo.orow : row;
    Sink sink(sp, l, srow, LAYOUT == 2 && row_beg < g0);
    const uint32_t scale = Sink::col_scale(sp);  // column deltas arrive multiplied by it
    const int S = (cnt + 3) >> 2;
    const int F = min(S - 1, cnt >> 2);  // steps j < F: four nonzeros and a next segment

    // stream offsets are 32-bit and wave-uniform (popcounts of ballots), so
    // they live in SGPRs
    uint32_t pos = cur.pos, dpos = cur.dpos, vpos = cur.vpos;
    const uint32_t *__restrict__ ED = cur.ED;
    const VT *__restrict__ EV = cur.EV;
    // A step's words: l1, l2 as loaded unless the check extracted them from
    // the state (e1, e2; then x1, x2), l3 always loaded.  The selection is
    // made at the top of the step that uses them, so that no instruction of
    // the step that loads them waits for those loads.
    uint32_t l1, l2, l3, x1 = 0, x2 = 0;
    bool e1 = false, e2 = false;
    {
        // lanes without a stream read a neighbouring word (buffers are padded)
        const uint64_t mk = ballot(S > 0);
        const uint32_t c = 4 * (uint32_t)__popcll(mk);
        l1 = src.read(pos, mk);
        l2 = src.read(pos + c, mk);
        l3 = src.read(pos + 2 * c, mk);
        pos += 3 * c;
        src.step_begin();
        src.consumed(pos);
    }
    const uint32_t pf = src.prefetch(pos, lane);
    uint32_t d = 0, r = 1, col = first_base(a.first_mode, (uint32_t)row) * scale;
    int64_t g = LAYOUT == 1 ? geo.gout : g0;

    auto step = [&](auto fullc, int j) {
        constexpr bool FULL = decltype(fullc)::value;
        const bool act = FULL || j < S;
        const bool more = FULL || j + 1 < S;
        const int rem = cnt - 4 * j;
        uint32_t od[4], ov[4];
        slot_offsets<(int)sizeof(VEntry<VT>)>(e1 ? x1 : l1, e2 ? x2 : l2, l3, od, ov);
        uint32_t dl[4], md[4], mv[4];
        VT v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t e = *(const uint64_t *)((const char *)tb.td + od[k]);
            const VEntry<VT> ve = *(const VEntry<VT> *)((const char *)tb.tv + ov[k]);
            dl[k] = (uint32_t)e;
            md[k] = (uint32_t)(e >> 32);
            v[k] = ve.value();
            mv[k] = ve.meta;
        }
        // Escapes (their loads issued before the next words, so that waiting
        // for them does not wait for the words): flagged by bit 31 of a slot's
        // metadata.  When no active lane has a flag in any of its eight
        // entries (the common case) nothing is masked; padding symbols are
        // never escapes, so only lanes past their last segment can hold one
        // otherwise.
        if constexpr (TF != 2) {
            const uint32_t fl = md[0] | md[1] | md[2] | md[3] | mv[0] | mv[1] | mv[2] | mv[3];
            if ((FULL ? ~0ull : ballot(act)) & ballot((int32_t)fl < 0)) {  // uniform
                if (a.esc_in_stream) {
                    // raw bits in the word stream at the read position:
                    // deltas, then values (FP64 as two words, low first),
                    // each nonzero position in lane order; the step's own
                    // words follow them
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const bool f = act && k < rem && (int32_t)md[k] < 0;
                        const uint64_t mk = ballot(f);
                        if (f) dl[k] = src.word_at(pos, 4 * lane_prefix(mk)) * scale;
                        pos += 4 * (uint32_t)__popcll(mk);
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const bool f = act && k < rem && (int32_t)mv[k] < 0;
                        const uint64_t mk = ballot(f);
                        if (f) {
                            const uint32_t o = (uint32_t)sizeof(VT) * lane_prefix(mk);
                            if constexpr (sizeof(VT) == 8) {
                                const uint64_t bits = (uint64_t)src.word_at(pos, o + 4) << 32 | src.word_at(pos, o);
                                v[k] = __builtin_bit_cast(VT, bits);
                            } else {
                                v[k] = __builtin_bit_cast(VT, src.word_at(pos, o));
                            }
                        }
                        pos += (uint32_t)sizeof(VT) * (uint32_t)__popcll(mk);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const bool f = act && k < rem && (int32_t)md[k] < 0;
                        const uint64_t mk = ballot(f);
                        if (f) dl[k] = ((gptr<uint32_t>)ED)[dpos + lane_prefix(mk)] * scale;
                        dpos += (uint32_t)__popcll(mk);
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const bool f = act && k < rem && (int32_t)mv[k] < 0;
                        const uint64_t mk = ballot(f);
                        if (f) v[k] = ((gptr<VT>)EV)[vpos + lane_prefix(mk)];
                        vpos += (uint32_t)__popcll(mk);
                    }
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    md[k] &= ~kMetaEscape;
                    mv[k] &= ~kMetaEscape;
                }
            }
        }
        // the two digit groups and their checks (Alg. 3), then the next
        // segment's words, in flight while this segment's x gathers are
        // served.  The loads are issued on every step, so that the wait
        // counts of the loads before them are the same on every path; lanes
        // that do not load (all of them on a wave's last step) read a
        // neighbouring word of the stream, whose value is not used.
        const uint64_t m3 = FULL ? ~0ull : ballot(more);  // lanes that load this step's words
        uint64_t m1 = 0, m2 = 0;
        if (FULL || m3) {
            uint32_t D, R;
            if constexpr (TF >= 1) {
                group_pairs(pair_rd(md[0], mv[0]), pair_rd(md[1], mv[1]), D, R);
                e1 = append_word(d, r, D, R, x1);
                group_pairs(pair_rd(md[2], mv[2]), pair_rd(md[3], mv[3]), D, R);
                e2 = append_word(d, r, D, R, x2);
            } else {
                group_general(md[0], mv[0], md[1], mv[1], D, R);
                e1 = append_and_check(d, r, D, R, x1);
                group_general(md[2], mv[2], md[3], mv[3], D, R);
                e2 = append_and_check(d, r, D, R, x2);
            }
            // masks combined on the scalar unit: a ballot of a plain compare
            // is the compare's own lane mask
            m1 = m3 & ~ballot(e1);
            m2 = m3 & ~ballot(e2);
        }
        {
            const uint32_t c1 = 4 * (uint32_t)__popcll(m1), c2 = 4 * (uint32_t)__popcll(m2);
            l1 = src.read(pos, m1);
            l2 = src.read(pos + c1, m2);
            if constexpr (FULL) {
                l3 = src.read_lanes(pos + c1 + c2, lane);
                pos += c1 + c2 + 4 * kWave;
            } else {
                l3 = src.read(pos + c1 + c2, m3);
                pos += c1 + c2 + 4 * (uint32_t)__popcll(m3);
            }
        }
        // deferred products of the previous step and the ring's pending chunk,
        // then the next chunk and this step's x loads, which the next step
        // waits for: a step waits on memory for loads issued a step earlier
        sink.pre_step();
        src.step_begin();
        src.consumed(pos);
        const int nreal = FULL ? 4 : (act ? min(rem, 4) : 0);
        uint32_t cols[4];
        int32_t rowk[4];
        if constexpr (LAYOUT == 1) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                col += dl[k];
                cols[k] = col;
                rowk[k] = srow;
            }
            // (the general-table decoder measured slower with paired loads)
            if constexpr (Sink::kPairs && TF == 0) sink.template segment<false, false>(cols, v, nreal, g, rowk);
            else sink.template segment<false>(cols, v, nreal, g, rowk);
        } else {
            // resolve row boundaries first: a column delta restarts at every
            // row; a nonzero at the end of the current row starts the next
            // nonempty one, whose predecessor the sink finishes
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < nreal && g + k >= row_end) {
                    ++krow;
                    row_beg = row_end;
                    row = n1.x;
                    row_end = n1.y;
                    n1 = n2;
                    n2 = a.nzr[min((int64_t)krow + 2, a.n_nzr)];
                    col = first_base(a.first_mode, (uint32_t)row) * scale;
                }
                col += dl[k];
                cols[k] = col;
                rowk[k] = row;
            }
            sink.template segment<true>(cols, v, nreal, g, rowk);
        }
        g += 4;
    };
    // full steps while every lane of the wavefront has one (a uniform test),
    // then the rest with per-lane masks
    int j = 0;
    if (ballot(0 < F) == ~0ull) {
        do {
            step(std::true_type(), j);
            ++j;
        } while (ballot(j < F) == ~0ull);
    }
    for (; ballot(j < S) != 0; ++j) step(std::false_type(), j);
    src.retire(pf);
    cur.pos = pos;
    cur.dpos = dpos;
    cur.vpos = vpos;
    if constexpr (LAYOUT == 1) {
        // (a cooperative sink needs every lane of the wavefront)
        if constexpr (Sink::kCoop) sink.finish_lane(srow, kComplete, live && l < a.m);
        else if (live && l < a.m) sink.finish_row(srow, kComplete);
    } else {
        // `row` holds this lane's last nonzeros: complete when it ends here;
        // started in an earlier lane, a head when it ends here, else a
        // middle; else a tail
        const int64_t gend = g0 + cnt;
        const bool ends = row_end <= gend;
        sink.finish_lane(row, row_beg < g0 ? (ends ? kHead : kMid) : (ends ? kComplete : kTail), live);
    }
}

// one encoded wave read straight from device memory
template <int LAYOUT, typename VT, class Sink, int TF>
__device__ __forceinline__ void decode_slice_global(const DevMat &a, const Tables<VT> &tb,
                                                    int64_t slice, uint32_t lane,
                                                    const typename Sink::Params &sp) {
    const uint64_t wo = uniform_load(a.woff + slice), we = uniform_load(a.woff + slice + 1);
    GlobalWords src{(const char *)(a.words + wo), 4 * (we - wo)};
    Cursor<VT> cur{0, 0, 0, a.escd + uniform_load(a.doff + slice),
                   (const VT *)a.escv + uniform_load(a.voff + slice)};
    const LaneGeo geo = lane_geo<LAYOUT>(a, slice, lane, lane_first_row<LAYOUT>(a, slice, lane));
    decode_slice<LAYOUT, VT, Sink, GlobalWords, TF>(a, tb, slice, lane, sp, src, cur, geo);
}

// Both tables into LDS in 16-byte pieces, every piece of a pass loaded before
// any is stored, so that a pass costs one memory round trip (two passes for a
// 1024-thread workgroup); the column deltas are multiplied by `scale` on the
// way (the sink's col_scale).
template <typename VT>
__device__ __forceinline__ void stage_tables(const DevMat &a, Tables<VT> &tb, uint32_t scale) {
    constexpr int kV = kSlots * (int)sizeof(VEntry<VT>) / 16, kT = kSlots * 8 / 16;
    constexpr int kAll = kV + kT, kU = 4;  // pieces per thread and pass
    const gptr<u32x4> gv = (gptr<u32x4>)a.tabval, gt = (gptr<u32x4>)a.tab;
    u32x4 *lds = (u32x4 *)&tb;  // tv, then td
    const int nt = blockDim.x;
    for (int b = 0; b < kAll; b += kU * nt) {
        u32x4 t[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int i = b + u * nt + (int)threadIdx.x;
            t[u] = u32x4{0u, 0u, 0u, 0u};
            if (i < kV) t[u] = gv[i];
            else if (i < kAll) {
                t[u] = gt[i - kV];
                t[u].x *= scale;  // two entries per piece: {delta, meta}, {delta, meta}
                t[u].z *= scale;
            }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int i = b + u * nt + (int)threadIdx.x;
            if (i < kAll) lds[i] = t[u];
        }
    }
    __syncthreads();
}

// Wave priority from the share of a wavefront's encoded waves still ahead of
// it (3 with more than three quarters left ... 0 in the last quarter).  The
// arbiter otherwise favours the oldest wavefronts, which then finish their
// (equal) shares early and leave the younger ones to end the launch at low
// occupancy; ranking by remaining work keeps the wavefronts of a CU in step.
// (The quarter is found by comparisons, not a 64-bit division, which would
// cost a hundred scalar instructions per wave.)
__device__ __forceinline__ void set_progress_priority(int64_t remaining, int64_t total) {
    const int64_t q = (remaining - 1) * 4;  // quarter = floor(q / total)
    if (total <= 0 || q < total) __builtin_amdgcn_s_setprio(0);
    else if (q < 2 * total) __builtin_amdgcn_s_setprio(1);
    else if (q < 3 * total) __builtin_amdgcn_s_setprio(2);
    else __builtin_amdgcn_s_setprio(3);
}

// The row-layout sweep of decode_kernel over waves s0, s0 + stride, ... below
// s_end (share of them).
// stage: 0 the tables are in LDS already; 1 stage them; 2 wait for the
// workgroup (its previous matrix), then stage them (the whole workgroup
// passes the same value).
template <typename VT, class Sink, int TF>
__device__ __forceinline__ void decode_rows(const DevMat &a, Tables<VT> &tb,
                                            uint32_t lane, const typename Sink::Params &sp,
                                            int64_t s_end, int64_t s0, int64_t stride,
                                            int64_t share, int stage = 1) {
    // Row layout: the next encoded wave's lane geometry and stream bases are
    // loaded while this one decodes, so a wave starts with one memory round
    // trip (its first words) instead of two; the first wave's are requested
    // before the tables are staged.  The loads for the next wave are issued
    // on every pass (past the last wave they read this wave's again), so that
    // no branch around them makes the wait counts of later loads unknown,
    // which would turn the first wait of the wave into a wait for everything
    // in flight.
    const int64_t sf = s0 < s_end ? s0 : a.num_waves - 1;  // in bounds for idle wavefronts
    LaneGeo geo = lane_geo<1>(a, sf, lane, lane_first_row<1>(a, sf, lane));
    uint64_t wo = uniform_load(a.woff + sf), we = uniform_load(a.woff + sf + 1);
    uint64_t dof = uniform_load(a.doff + sf), vof = uniform_load(a.voff + sf);
    if (stage == 2) __syncthreads();
    if (stage) stage_tables<VT>(a, tb, Sink::col_scale(sp));
    int64_t k = 0;
    for (int64_t s = s0; s < s_end; s += stride, ++k) {
        const int64_t s1 = s + stride < s_end ? s + stride : s;
        const LaneGeo next = lane_geo<1>(a, s1, lane, lane_first_row<1>(a, s1, lane));
        const uint64_t wo1 = uniform_load(a.woff + s1), we1 = uniform_load(a.woff + s1 + 1);
        const uint64_t dof1 = uniform_load(a.doff + s1), vof1 = uniform_load(a.voff + s1);
        GlobalWords src{(const char *)(a.words + wo), 4 * (we - wo)};
        Cursor<VT> cur{0, 0, 0, a.escd + dof, (const VT *)a.escv + vof};
        set_progress_priority(share - k, share);
        decode_slice<1, VT, Sink, GlobalWords, TF>(a, tb, s, lane, sp, src, cur, geo);
        geo = next;
        wo = wo1;
        we = we1;
        dof = dof1;
        vof = vof1;
    }
}

// The sweep of one persistent workgroup over its encoded waves (tables
// staged into LDS on the way).
template <int LAYOUT, typename VT, class Sink, int TF>
__device__ __forceinline__ void decode_sweep(const DevMat &a, const typename Sink::Params &sp,
                                             Tables<VT> &tb) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const int64_t wpb = blockDim.x / kWave;
    const int64_t total = (int64_t)gridDim.x * wpb;
    // Workgroups are dispatched round-robin over the XCDs.  The workgroups of
    // one XCD own one contiguous share of the encoded waves, and their
    // wavefronts sweep it together (wavefront i takes waves i, i + W, ...), so
    // at any time an XCD decodes a compact window of rows and its x gathers
    // stay in that XCD's L2.  The wave index is uniform (readfirstlane).
    const int64_t G = gridDim.x, xcd = blockIdx.x % kNumXcd, pos_in_xcd = blockIdx.x / kNumXcd;
    const int64_t q = G / kNumXcd, rr = G % kNumXcd;
    const int64_t xcd_blocks = q + (xcd < rr ? 1 : 0);
    const int64_t xcd_first = xcd * q + (xcd < rr ? xcd : rr);
    const int64_t s_begin = xcd_first * wpb * a.num_waves / total;
    const int64_t s_end = (xcd_first + xcd_blocks) * wpb * a.num_waves / total;
    const int64_t stride = xcd_blocks * wpb;
    const int64_t s0 = s_begin + pos_in_xcd * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t share = s0 < s_end ? (s_end - 1 - s0) / stride + 1 : 0;  // encoded waves of this wavefront
    if constexpr (LAYOUT == 2) {
        stage_tables<VT>(a, tb, Sink::col_scale(sp));
        // long lanes: a wave's start-up is a small part of its work
        for (int64_t s = s0, k = 0; s < s_end; s += stride, ++k) {
            set_progress_priority(share - k, share);
            decode_slice_global<LAYOUT, VT, Sink, TF>(a, tb, s, lane, sp);
        }
    } else {
        decode_rows<VT, Sink, TF>(a, tb, lane, sp, s_end, s0, stride, share);
    }
}

// MINW: waves per SIMD the register allocation must allow (8 lets two
// 16-wave workgroups share a CU, which is what the LDS tables permit).  Below
// 4 the workgroup is capped at 4 * MINW waves, so that the compiler may give
// a wave more than 128 registers.
constexpr int decode_max_threads(int minw) { return minw >= 4 ? 1024 : 256 * minw; }
template <int LAYOUT, typename VT, class Sink, int MINW, int TF>
__global__ __launch_bounds__(decode_max_threads(MINW), MINW) void decode_kernel(DevMat a, typename Sink::Params sp) {
    __shared__ __align__(16) Tables<VT> tb;
    decode_sweep<LAYOUT, VT, Sink, TF>(a, sp, tb);
}

// Transposed product with dX privatised in LDS: a workgroup (one per CU)
// scatters into its own copy of the n x KC block of dX with LDS atomic adds,
// then writes it to part[blockIdx.x]; trans_reduce_kernel sums the copies.
// No global atomics, so no contention when n is small (the tall pruned
// weight: every column of dX receives thousands of contributions).
template <int LAYOUT, typename VT, int KC, int TF>
__global__ __launch_bounds__(1024, 4) void trans_lds_kernel(DevMat a,
                                                            typename TransLdsSink<VT, KC>::Params sp,
                                                            VT *part) {
    __shared__ __align__(16) Tables<VT> tb;
    extern __shared__ __align__(16) unsigned char s_dyn[];
    VT *s_dx = (VT *)s_dyn;
    const int64_t cnt = a.n * KC, slots = lds_slot((uint32_t)cnt);
    for (int64_t i = threadIdx.x; i < slots; i += blockDim.x) s_dx[i] = (VT)0;
    // (the table staging inside the sweep ends with a barrier, which also
    // orders these stores before the first scatter)
    typename TransLdsSink<VT, KC>::Params q = sp;
    q.lds = s_dx;
    decode_sweep<LAYOUT, VT, TransLdsSink<VT, KC>, TF>(a, q, tb);
    __syncthreads();
    VT *dst = part + (int64_t)blockIdx.x * cnt;
    for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) dst[i] = s_dx[lds_slot((uint32_t)i)];
}

// dX (KC columns) = alpha * (sum of the G copies) + beta * dX
template <typename VT>
__global__ __launch_bounds__(256) void trans_reduce_kernel(const VT *part, int64_t G, int64_t n,
                                                           int KC, VT *dX, int64_t lddx,
                                                           double alpha, double beta) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, cnt = n * KC;
    if (i >= cnt) return;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // eight loads in flight
    int64_t b = 0;
    for (; b + 8 <= G; b += 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += (double)part[(b + u) * cnt + i];
    for (; b < G; ++b) acc[0] += (double)part[b * cnt + i];
    const double sum = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    VT *d = dX + (i / KC) * lddx + i % KC;
    *d = (VT)(beta == 0.0 ? alpha * sum : alpha * sum + beta * (double)*d);
}

// Same work as decode_kernel, with every wavefront owning one contiguous run
// of encoded waves (so that its streams are adjacent in memory) and reading
// them through an LDS ring (RingWords).  The XCD shares are those of
// decode_kernel; inside a share the runs are consecutive, which keeps the
// rows an XCD works on within a window of its share.
template <int LAYOUT, typename VT, class Sink, int MINW, int TF>
__global__ __launch_bounds__(1024, MINW) void ring_kernel(DevMat a, typename Sink::Params sp) {
    __shared__ __align__(16) Tables<VT> tb;
    extern __shared__ uint32_t s_ring[];  // RingWords<kRingWords>::kWords per wavefront
    stage_tables<VT>(a, tb, Sink::col_scale(sp));
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const int64_t wpb = blockDim.x / kWave;
    const int64_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t G = gridDim.x, xcd = blockIdx.x % kNumXcd, pos_in_xcd = blockIdx.x / kNumXcd;
    const int64_t q = G / kNumXcd, rr = G % kNumXcd;
    const int64_t xcd_blocks = q + (xcd < rr ? 1 : 0);
    const int64_t xcd_first = xcd * q + (xcd < rr ? xcd : rr);
    const int64_t total = G * wpb;
    const int64_t s_begin = xcd_first * wpb * a.num_waves / total;
    const int64_t s_end = (xcd_first + xcd_blocks) * wpb * a.num_waves / total;
    const int64_t nw = xcd_blocks * wpb, widx = pos_in_xcd * wpb + wib;
    const int64_t sa = s_begin + widx * (s_end - s_begin) / nw;
    const int64_t sb = s_begin + (widx + 1) * (s_end - s_begin) / nw;
    if (sa >= sb) return;
    RingWords<kRingWords> src;
    const uint64_t w0 = a.woff[sa];
    src.start(s_ring + wib * RingWords<kRingWords>::kWords, a.words + w0,
              (uint32_t)(4 * (a.woff[sb] - w0)), lane);
    Cursor<VT> cur{0, 0, 0, a.escd + a.doff[sa], (const VT *)a.escv + a.voff[sa]};
    // lane geometry two stages ahead: first rows of wave s + 2 and row
    // pointers of wave s + 1 are loaded while wave s decodes
    LaneGeo geo = lane_geo<LAYOUT>(a, sa, lane, lane_first_row<LAYOUT>(a, sa, lane));
    int32_t fr1 = sa + 1 < sb ? lane_first_row<LAYOUT>(a, sa + 1, lane) : 0;
    for (int64_t s = sa; s < sb; ++s) {
        const int32_t fr2 = s + 2 < sb ? lane_first_row<LAYOUT>(a, s + 2, lane) : 0;
        LaneGeo next{0, 0, 0, 0, 0, 0};
        if (s + 1 < sb) next = lane_geo<LAYOUT>(a, s + 1, lane, fr1);
        decode_slice<LAYOUT, VT, Sink, RingWords<kRingWords>, TF>(a, tb, s, lane, sp, src, cur, geo);
        geo = next;
        fr1 = fr2;
    }
}

// rows split over lanes (layout NNZ): y = alpha * (tail of the first lane +
// heads of the following lanes) + beta * y.  A row spanning at most
// kLongSplit (kLongSplitRuns) following lanes is summed by one thread
// (fixup_kernel); a longer one by a whole wavefront (fixup_long_kernel, rows
// listed on the host): its lanes stride over the row's partials, one running
// sum per column, then a butterfly reduction per column.
constexpr int kMaxFixupCols = 32;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <typename VT>
__device__ __forceinline__ void fixup_put(VT *Y, int64_t ldy, int32_t row, int c, double sum,
                                          double alpha, double beta) {
    VT *y = Y + (int64_t)row * ldy + c;
    *y = (VT)(beta == 0.0 ? alpha * sum : alpha * sum + beta * (double)*y);
}

// runs: the middle lanes' pieces were summed per wavefront (finish_lane), so
// of the lanes strictly between the first (a) and the last (b) only the one
// after the first and those starting a wavefront hold a partial; the first
// wavefront start after a + 1:
__device__ __forceinline__ int64_t first_run_start(int32_t a) { return ((int64_t)(a + 1) | (kWave - 1)) + 1; }

template <typename VT>
__global__ __launch_bounds__(256) void fixup_kernel(SplitRows sr, const double *partial, int KC,
                                                    int runs, VT *Y, int64_t ldy, double alpha,
                                                    double beta, int log_tpr) {
    // 2^log_tpr >= KC threads per split row, one column each (consecutive
    // threads read consecutive doubles of a partial slot)
    const int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> log_tpr;
    const int c = (int)(threadIdx.x & ((1u << log_tpr) - 1));
    if (s >= sr.n || c >= KC) return;
    const int32_t a = sr.first[s], b = sr.last[s];
    if (b - a > (runs ? kLongSplitRuns : kLongSplit)) return;
    {
        const double *head = partial + c;  // head slot of lane l: head[2 * l * KC]
        double sum = partial[(2 * (int64_t)a + 1) * KC + c];
        if (runs) {
            sum += head[2 * (int64_t)(a + 1) * KC];
            for (int64_t l = first_run_start(a); l < b; l += kWave) sum += head[2 * l * KC];
            if (b > a + 1) sum += head[2 * (int64_t)b * KC];
        } else {
            for (int64_t l = a + 1; l <= b; ++l) sum += head[2 * l * KC];
        }
        fixup_put(Y, ldy, sr.row[s], c, sum, alpha, beta);
    }
}

template <typename VT>
__global__ __launch_bounds__(256) void fixup_long_kernel(SplitRows sr, const double *partial, int KC,
                                                         int runs, VT *Y, int64_t ldy, double alpha,
                                                         double beta) {
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = (int)(threadIdx.x & (kWave - 1));
    if (w >= sr.n_long) return;  // whole wavefronts
    const int64_t s = sr.longs[w];
    const int32_t a = sr.first[s], b = sr.last[s];
    double acc[kMaxFixupCols];
#pragma unroll
    for (int c = 0; c < kMaxFixupCols; ++c) acc[c] = 0.0;
    auto add = [&](const double *q) {
#pragma unroll
        for (int c = 0; c < kMaxFixupCols; ++c)
            if (c < KC) acc[c] += q[c];
    };
    if (runs) {
        // lane 0: the tail of lane a and the head of lane a + 1; lane 1: the
        // head of lane b; all lanes: the wavefront starts in between
        if (lane == 0) {
            add(partial + (2 * (int64_t)a + 1) * KC);
            add(partial + 2 * (int64_t)(a + 1) * KC);
        }
        if (lane == 1) add(partial + 2 * (int64_t)b * KC);
        for (int64_t l = first_run_start(a) + (int64_t)lane * kWave; l < b; l += (int64_t)kWave * kWave)
            add(partial + 2 * l * KC);
    } else {
        for (int64_t l = (int64_t)a + lane; l <= b; l += kWave)
            add(partial + (2 * l + (l == a ? 1 : 0)) * KC);  // tail of lane a, heads after
    }
#pragma unroll
    for (int c = 0; c < kMaxFixupCols; ++c)
        if (c < KC) {
            const double sum = wave_sum(acc[c]);
            if (lane == c) fixup_put(Y, ldy, sr.row[s], c, sum, alpha, beta);
        }
}

// both fix-up kernels for KC <= kMaxFixupCols columns of Y
template <typename VT>
hipError_t launch_fixup(const SplitRows &sr, const double *partial, int KC, int runs, VT *Y,
                        int64_t ldy, double alpha, double beta, hipStream_t st) {
    if (sr.n == 0) return hipSuccess;
    if (KC > kMaxFixupCols) return hipErrorInvalidValue;
    int lt = 0;
    while ((1 << lt) < KC) ++lt;
    const int64_t threads = sr.n << lt;
    hipLaunchKernelGGL(fixup_kernel<VT>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, sr,
                       partial, KC, runs, Y, ldy, alpha, beta, lt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || sr.n_long == 0) return e;
    hipLaunchKernelGGL(fixup_long_kernel<VT>, dim3((unsigned)((sr.n_long + 3) / 4)), dim3(256), 0, st,
                       sr, partial, KC, runs, Y, ldy, alpha, beta);
    return hipGetLastError();
}

// Y[rows, :KC] = beta * Y (beta == 0: zero)
template <typename VT>
__global__ void scale_kernel(VT *Y, int64_t rows, int KC, int64_t ldy, double beta) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * KC) return;
    VT *y = Y + (i / KC) * ldy + i % KC;
    *y = beta == 0.0 ? (VT)0 : (VT)(beta * (double)*y);
}

__global__ __launch_bounds__(256) void flush_kernel(const uint4 *p, int64_t n, uint32_t *sink) {
    uint32_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint4 v = p[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;  // keeps the loads; the buffer is zero
}

// layout NNZ: y = beta * y on the rows without nonzeros (never decoded)
template <typename VT>
__global__ void empty_rows_kernel(const int32_t *rows, int64_t count, VT *Y, int KC, int64_t ldy,
                                  double beta) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count * KC) return;
    VT *y = Y + (int64_t)rows[i / KC] * ldy + i % KC;
    *y = beta == 0.0 ? (VT)0 : (VT)(beta * (double)*y);
}

// ------------------------------------------------- multi-matrix launch
template <typename VT>
__global__ __launch_bounds__(1024, 7) void batch_kernel(BatchDev b, double alpha, double beta) {
    __shared__ __align__(16) Tables<VT> tb;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), wpb = blockDim.x / kWave;
    const int t0 = b.wg_task[blockIdx.x], t1 = b.wg_task[blockIdx.x + 1];
    int cur = -1;
    for (int t = t0; t < t1; ++t) {
        const BatchTask task = b.tasks[t];
        const DevMat a = b.mats[task.mat];  // uniform: scalar loads into SGPRs
        // the tables are restaged only when the matrix changes
        const int stage = task.mat == cur ? 0 : (cur < 0 ? 1 : 2);
        cur = task.mat;
        typename SpmmSink<VT, 1, true>::Params sp;
        sp.X = (const VT *)b.ptrs[2 * task.mat];
        sp.ldx = 1;
        sp.Y = (VT *)b.ptrs[2 * task.mat + 1];
        sp.ldy = 1;
        sp.partial = nullptr;
        sp.alpha = alpha;
        sp.beta = beta;
        sp.pair_x = a.n >= 2;
        // this wavefront's waves of the task: first_wave + wib, + wpb, ...
        const int64_t s0 = task.first_wave + wib, s_end = (int64_t)task.first_wave + task.num_waves;
        const int64_t share = s0 < s_end ? (s_end - 1 - s0) / wpb + 1 : 0;
        if (a.base_direct)
            decode_rows<VT, SpmmSink<VT, 1, true>, 1>(a, tb, lane, sp, s_end, s0, wpb, share, stage);
        else
            decode_rows<VT, SpmmSink<VT, 1, true>, 0>(a, tb, lane, sp, s_end, s0, wpb, share, stage);
    }
}

// The same launch for k right-hand sides: X_i is n_i x k and Y_i m_i x k, row
// major with leading dimension k; this launch takes the columns c0 .. c0 + KC
// of every matrix (the sink's chunk), each matrix decoded once per launch.
template <typename VT, class Sink, int MINW>
__global__ __launch_bounds__(decode_max_threads(MINW), MINW) void batch_spmm_kernel(BatchDev b, int c0, int k,
                                                                                     double alpha, double beta) {
    __shared__ __align__(16) Tables<VT> tb;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), wpb = blockDim.x / kWave;
    const int t0 = b.wg_task[blockIdx.x], t1 = b.wg_task[blockIdx.x + 1];
    int cur = -1;
    for (int t = t0; t < t1; ++t) {
        const BatchTask task = b.tasks[t];
        const DevMat a = b.mats[task.mat];
        const int stage = task.mat == cur ? 0 : (cur < 0 ? 1 : 2);
        cur = task.mat;
        typename Sink::Params sp;
        sp.X = (const VT *)b.ptrs[2 * task.mat] + c0;
        sp.ldx = (uint32_t)k;
        sp.Y = (VT *)b.ptrs[2 * task.mat + 1] + c0;
        sp.ldy = (uint32_t)k;
        sp.partial = nullptr;  // row layout: every row ends in its lane
        sp.alpha = alpha;
        sp.beta = beta;
        const int64_t s0 = task.first_wave + wib, s_end = (int64_t)task.first_wave + task.num_waves;
        const int64_t share = s0 < s_end ? (s_end - 1 - s0) / wpb + 1 : 0;
        if (a.base_direct)
            decode_rows<VT, Sink, 1>(a, tb, lane, sp, s_end, s0, wpb, share, stage);
        else
            decode_rows<VT, Sink, 0>(a, tb, lane, sp, s_end, s0, wpb, share, stage);
    }
}

// ------------------------------------------------------- plain CSR
// variant 1: G lanes per row (G a power of two <= 64), lanes of a group read
// consecutive nonzeros; butterfly reduction inside the group.
template <typename VT, int G, int KC>
__global__ __launch_bounds__(256) void csr_vector_kernel(CsrDev c, const VT *__restrict__ X,
                                                         int64_t ldx, VT *__restrict__ Y,
                                                         int64_t ldy, double alpha, double beta) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const int q = threadIdx.x % G;
    const VT *__restrict__ val = (const VT *)c.val;
    for (int64_t row = tid / G; row < c.m; row += nthreads / G) {
        const int32_t b = c.row_ptr[row], e = c.row_ptr[row + 1];
        double acc[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) acc[k] = 0.0;
        for (int32_t i = b + q; i < e; i += G) {
            const VT v = val[i];
            const VT *x = X + (int64_t)c.col[i] * ldx;
#pragma unroll
            for (int k = 0; k < KC; ++k) acc[k] = fma((double)v, (double)x[k], acc[k]);
        }
#pragma unroll
        for (int k = 0; k < KC; ++k) {
#pragma unroll
            for (int off = G / 2; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, G);
        }
        if (q == 0) {
            VT *y = Y + row * ldy;
#pragma unroll
            for (int k = 0; k < KC; ++k)
                y[k] = (VT)(beta == 0.0 ? alpha * acc[k] : alpha * acc[k] + beta * (double)y[k]);
        }
    }
}

// variant 2: lane_nnz consecutive nonzeros per lane, rows tracked through
// row_ptr, partial sums of rows that cross lanes go to `partial`.
template <typename VT, int KC>
__global__ __launch_bounds__(256) void csr_split_kernel(CsrDev c, const VT *__restrict__ X,
                                                        int64_t ldx, VT *__restrict__ Y,
                                                        int64_t ldy, double alpha, double beta,
                                                        double *partial) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= c.num_lanes) return;
    const VT *__restrict__ val = (const VT *)c.val;
    const int64_t g0 = l * (int64_t)c.lane_nnz;
    const int64_t gend = min(g0 + c.lane_nnz, c.nnz);
    int32_t row = c.lane_row[l];
    int32_t row_beg = c.row_ptr[row], row_end = c.row_ptr[row + 1];
    double acc[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) acc[k] = 0.0;
    auto done = [&](int kind) {
        if (kind == kComplete) {
            VT *y = Y + (int64_t)row * ldy;
#pragma unroll
            for (int k = 0; k < KC; ++k)
                y[k] = (VT)(beta == 0.0 ? alpha * acc[k] : alpha * acc[k] + beta * (double)y[k]);
        } else {
            double *q = partial + (2 * l + (kind == kTail ? 1 : 0)) * KC;
#pragma unroll
            for (int k = 0; k < KC; ++k) q[k] = acc[k];
        }
#pragma unroll
        for (int k = 0; k < KC; ++k) acc[k] = 0.0;
    };
    for (int64_t g = g0; g < gend; ++g) {
        while (g >= row_end) {
            done(row_beg < g0 ? kHead : kComplete);
            ++row;
            row_beg = row_end;
            row_end = c.row_ptr[row + 1];
        }
        const VT v = val[g];
        const VT *x = X + (int64_t)c.col[g] * ldx;
#pragma unroll
        for (int k = 0; k < KC; ++k) acc[k] = fma((double)v, (double)x[k], acc[k]);
    }
    while (row < c.m && row_end <= gend) {
        done(row_beg < g0 ? kHead : kComplete);
        ++row;
        row_beg = row_end;
        if (row < c.m) row_end = c.row_ptr[row + 1];
    }
    if (row < c.m && row_beg < gend) done(row_beg < g0 ? kHead : kTail);
}

// variant 3 (SpMV): CSR-stream.  A workgroup takes a block of consecutive
// rows holding at most kStreamNnz nonzeros, loads their column indices and
// values coalesced (four per thread, all x gathers in flight together),
// stages the products in LDS and sums each row from LDS.  A block that is a
// single row longer than that is reduced across the workgroup instead.
constexpr int kStreamNnz = 1024;
template <typename VT>
__global__ __launch_bounds__(256) void csr_stream_kernel(CsrDev c, const int32_t *__restrict__ blk,
                                                         const VT *__restrict__ x, VT *__restrict__ y,
                                                         double alpha, double beta) {
    __shared__ double prod[kStreamNnz];
    __shared__ double red[4];
    const int r0 = blk[blockIdx.x], r1 = blk[blockIdx.x + 1];
    const int32_t g0 = c.row_ptr[r0], g1 = c.row_ptr[r1];
    const VT *__restrict__ val = (const VT *)c.val;
    const int32_t *__restrict__ col = c.col;
    const int tid = threadIdx.x;
    if (g1 - g0 > kStreamNnz) {  // one long row
        double s = 0.0;
        for (int32_t base = g0; base < g1; base += 4 * 256) {
            VT v[4], xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int32_t i = base + u * 256 + tid;
                v[u] = i < g1 ? val[i] : (VT)0;
                xv[u] = i < g1 ? x[col[i]] : (VT)0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) s = fma((double)v[u], (double)xv[u], s);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if ((tid & 63) == 0) red[tid >> 6] = s;
        __syncthreads();
        if (tid == 0) {
            const double t = red[0] + red[1] + red[2] + red[3];
            y[r0] = (VT)(beta == 0.0 ? alpha * t : alpha * t + beta * (double)y[r0]);
        }
        return;
    }
    const int32_t cnt = g1 - g0;
    VT v[4], xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int32_t i = u * 256 + tid;
        if (i < cnt) {
            v[u] = val[g0 + i];
            xv[u] = x[col[g0 + i]];
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int32_t i = u * 256 + tid;
        if (i < cnt) prod[i] = (double)v[u] * (double)xv[u];
    }
    __syncthreads();
    for (int r = r0 + tid; r < r1; r += 256) {
        const int32_t b = c.row_ptr[r] - g0, e = c.row_ptr[r + 1] - g0;
        double s = 0.0;
        for (int32_t i = b; i < e; ++i) s += prod[i];
        y[r] = (VT)(beta == 0.0 ? alpha * s : alpha * s + beta * (double)y[r]);
    }
}

// ------------------------------------------------------------ dispatch
template <class T> struct TypeBox { typedef T type; };

// the nonzero-balanced layout tracks rows and needs a few more registers
constexpr int occ_nnz(int occ) { return occ > 7 ? 7 : occ; }

template <typename F>
hipError_t for_kc(int k, int kcmax, F f);
template <typename F>
hipError_t for_kc(int k, F f) {
    return for_kc(k, kMaxPassCols, f);
}
template <typename F>
hipError_t for_kc(int k, int kcmax, F f) {
    // split k columns into compile-time chunks of at most kcmax
    int c0 = 0;
    while (c0 < k) {
        int left = k - c0 < kcmax ? k - c0 : kcmax;
        hipError_t e;
        if (left >= 32) { e = f(std::integral_constant<int, 32>(), c0); c0 += 32; }
        else if (left >= 16) { e = f(std::integral_constant<int, 16>(), c0); c0 += 16; }
        else if (left >= 8) { e = f(std::integral_constant<int, 8>(), c0); c0 += 8; }
        else if (left >= 4) { e = f(std::integral_constant<int, 4>(), c0); c0 += 4; }
        else if (left >= 2) { e = f(std::integral_constant<int, 2>(), c0); c0 += 2; }
        else { e = f(std::integral_constant<int, 1>(), c0); c0 += 1; }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// layout NNZ after the decode: rows split over lanes, then rows without
// nonzeros (both only write y)
template <typename VT>
hipError_t nnz_epilogue(const DevMat &a, const double *partial, int KC, VT *Y, int64_t ldy,
                        double alpha, double beta, hipStream_t st) {
    hipError_t e = launch_fixup(a.split, partial, KC, 1, Y, ldy, alpha, beta, st);
    if (e != hipSuccess) return e;
    if (a.n_empty > 0) {
        const int64_t tot = a.n_empty * KC;
        hipLaunchKernelGGL(empty_rows_kernel<VT>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                           a.empty_rows, a.n_empty, Y, KC, ldy, beta);
        return hipGetLastError();
    }
    return hipSuccess;
}

// the kernel instance for the matrix's table format
template <typename K>
K pick_bd(const DevMat &a, K direct, K general) {
    return a.base_direct ? direct : general;
}
template <typename K>
K pick_tf(const DevMat &a, K direct_noesc, K direct, K general) {
    return a.base_direct ? (a.no_escape ? direct_noesc : direct) : general;
}

// Launch of a persistent direct-read decode kernel.  Unless the caller fixed
// the shape, the workgroup size (16, 12, 8 or 4 waves: multiples of the
// CU's 4 SIMDs) is the one that keeps the most wavefronts resident according
// to the runtime's occupancy for this kernel, whose registers and LDS both
// limit it (a 12-wave workgroup of a kernel that fits 4 waves per SIMD would
// leave a CU with one workgroup, 3 waves per SIMD); cached per kernel.
struct Shape {
    int wpw, per_cu;
};
template <typename K>
Shape fit_shape(K kern, const Launch &L) {
    // the occupancy query does not know the kernel's workgroup-size bound, and
    // a fixed shape may exceed it (kernels that need more than 128 registers)
    auto max_threads = [&]() {
        hipFuncAttributes fa;
        return hipFuncGetAttributes(&fa, (const void *)kern) == hipSuccess ? fa.maxThreadsPerBlock : 1024;
    };
    if (L.fixed_shape)
        return Shape{std::min(L.waves_per_wg, max_threads() / 64), std::max(1, (L.grid + L.num_cus - 1) / L.num_cus)};
    static std::mutex mu;
    static std::vector<std::pair<const void *, Shape>> cache;
    const void *key = (const void *)kern;
    std::lock_guard<std::mutex> lock(mu);
    for (const auto &c : cache)
        if (c.first == key) return c.second;
    const int mt = max_threads();
    Shape best{L.waves_per_wg, std::max(1, (L.grid + L.num_cus - 1) / L.num_cus)};
    int best_res = 0;
    for (int w : {16, 12, 8, 4}) {
        int nb = 0;
        if (64 * w > mt) continue;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, 64 * w, 0) != hipSuccess) continue;
        if (nb * w > best_res) {
            best_res = nb * w;
            best = Shape{w, nb};
        }
    }
    cache.emplace_back(key, best);
    return best;
}

template <typename K, typename... Args>
hipError_t launch_persistent(K kern, const DevMat &a, const Launch &L, hipStream_t st, Args... args) {
    const Shape sh = fit_shape(kern, L);
    const int64_t need = (a.num_waves + sh.wpw - 1) / sh.wpw;
    const int64_t grid = L.fixed_shape ? L.grid : std::min<int64_t>((int64_t)L.num_cus * sh.per_cu, need);
    hipLaunchKernelGGL(kern, dim3((unsigned)std::max<int64_t>(1, grid)), dim3(64 * sh.wpw), 0, st, args...);
    return hipGetLastError();
}

template <typename VT>
hipError_t spmm_impl(const DevMat &a, int k, const VT *X, int64_t ldx, VT *Y, int64_t ldy,
                     double alpha, double beta, double *partial, Launch L, hipStream_t st) {
    if (a.nnz == 0 || a.num_waves == 0) {
        if (a.m == 0) return hipSuccess;
        return for_kc(k, [&](auto KCc, int c0) {
            constexpr int KC = decltype(KCc)::value;
            int64_t tot = a.m * KC;
            hipLaunchKernelGGL(scale_kernel<VT>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                               st, Y + c0, a.m, KC, ldy, beta);
            return hipGetLastError();
        });
    }
    auto launch = [&](auto sinkc, int KC, int c0) -> hipError_t {
        typedef typename decltype(sinkc)::type SinkT;
        typename SinkT::Params sp;
        sp.X = X + c0;
        sp.ldx = (uint32_t)ldx;
        sp.Y = Y + c0;
        sp.ldy = (uint32_t)ldy;
        sp.partial = partial;
        sp.alpha = alpha;
        sp.beta = beta;
        hipError_t e = a.layout == 1
                           ? launch_persistent(pick_bd(a, decode_kernel<1, VT, SinkT, SinkT::kOcc, 1>,
                                                       decode_kernel<1, VT, SinkT, SinkT::kOcc, 0>),
                                               a, L, st, a, sp)
                           : launch_persistent(pick_bd(a, decode_kernel<2, VT, SinkT, occ_nnz(SinkT::kOcc), 1>,
                                                       decode_kernel<2, VT, SinkT, occ_nnz(SinkT::kOcc), 0>),
                                               a, L, st, a, sp);
        if (e != hipSuccess || a.layout != 2) return e;
        return nnz_epilogue(a, partial, KC, Y + c0, ldy, alpha, beta, st);
    };
    // LDS-ring kernels: deferred products, at most 2 (FP64) / 4 (FP32) columns
    // per pass so that the deferred x values stay in registers
    auto ring = [&](auto sinkc, auto kern, int KC, int c0) -> hipError_t {
        typedef typename decltype(sinkc)::type SinkT;
        typename SinkT::Params sp;
        sp.X = X + c0;
        sp.ldx = (uint32_t)ldx;
        sp.Y = Y + c0;
        sp.ldy = (uint32_t)ldy;
        sp.partial = partial;
        sp.alpha = alpha;
        sp.beta = beta;
        const int rw = L.ring_waves_per_wg;
        const dim3 rblock(64 * rw);
        const size_t lds = (size_t)rw * RingWords<kRingWords>::kWords * 4;
        int per_cu = L.wg_per_cu;
        if (per_cu <= 0) {
            hipError_t e = hipFuncSetAttribute((const void *)kern,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, (int)rblock.x, lds);
            if (e != hipSuccess) return e;
            per_cu = per_cu > 0 ? per_cu : 1;
        }
        const int64_t need = (a.num_waves + rw - 1) / rw;
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)L.num_cus * per_cu, need));
        hipLaunchKernelGGL(kern, dim3(grid), rblock, lds, st, a, sp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || a.layout != 2) return e;
        return nnz_epilogue(a, partial, KC, Y + c0, ldy, alpha, beta, st);
    };
    const bool unit = k == 1 && ldx == 1 && ldy == 1 && a.n * (int64_t)sizeof(VT) <= (1ll << 32);
    if (L.ring) {
        if (unit) {
            typedef SpmmSink<VT, 1, true, double, 1> RowSink;
            typedef SpmmSink<VT, 1, true, double, 2> NnzSink;
            if (a.layout == 1)
                return ring(TypeBox<RowSink>(), pick_bd(a, ring_kernel<1, VT, RowSink, 4, 1>,
                                                        ring_kernel<1, VT, RowSink, 4, 0>), 1, 0);
            return ring(TypeBox<NnzSink>(), pick_bd(a, ring_kernel<2, VT, NnzSink, 4, 1>,
                                                    ring_kernel<2, VT, NnzSink, 4, 0>), 1, 0);
        }
        return for_kc(k, std::is_same<VT, double>::value ? 2 : 4, [&](auto KCc, int c0) {
            constexpr int KC = decltype(KCc)::value;
            if constexpr (KC > 4 || (std::is_same<VT, double>::value && KC > 2)) {
                return hipErrorInvalidValue;  // excluded by the chunk limit
            } else {
                typedef SpmmSink<VT, KC, false, double, 1> RowSink;
                typedef SpmmSink<VT, KC, false, double, 2> NnzSink;
                if (a.layout == 1)
                    return ring(TypeBox<RowSink>(), pick_bd(a, ring_kernel<1, VT, RowSink, 4, 1>,
                                                            ring_kernel<1, VT, RowSink, 4, 0>),
                                KC, c0);
                return ring(TypeBox<NnzSink>(), pick_bd(a, ring_kernel<2, VT, NnzSink, 4, 1>,
                                                        ring_kernel<2, VT, NnzSink, 4, 0>),
                            KC, c0);
            }
        });
    }
    if (unit) {
        // single vectors also have instances without escape handling
        typedef SpmmSink<VT, 1, true> SinkT;
        typename SinkT::Params sp;
        sp.X = X;
        sp.ldx = 1;
        sp.Y = Y;
        sp.ldy = 1;
        sp.partial = partial;
        sp.alpha = alpha;
        sp.beta = beta;
        sp.pair_x = a.n >= 2;
        constexpr int occ = SinkT::kOcc, occn = occ_nnz(SinkT::kOcc);
        hipError_t e =
            a.layout == 1
                ? launch_persistent(pick_tf(a, decode_kernel<1, VT, SinkT, occ, 2>, decode_kernel<1, VT, SinkT, occ, 1>,
                                            decode_kernel<1, VT, SinkT, occ, 0>),
                                    a, L, st, a, sp)
                : launch_persistent(pick_tf(a, decode_kernel<2, VT, SinkT, occn, 2>, decode_kernel<2, VT, SinkT, occn, 1>,
                                            decode_kernel<2, VT, SinkT, occn, 0>),
                                    a, L, st, a, sp);
        if (e != hipSuccess || a.layout != 2) return e;
        return nnz_epilogue(a, partial, 1, Y, ldy, alpha, beta, st);
    }
    // Several columns: groups of lanes share each row of X (CoopSpmmSink) when
    // its rows can be read as aligned 16-byte pieces at 32-bit byte offsets;
    // chunks of 32 / 16 / 8 FP32 or 16 / 8 / 4 FP64 columns, the rest as below.
    const bool coop = (uintptr_t)X % 16 == 0 && (ldx * (int64_t)sizeof(VT)) % 16 == 0 &&
                      a.n * ldx * (int64_t)sizeof(VT) <= (1ll << 32);
    if (coop) {
        constexpr int CLv = 16 / (int)sizeof(VT);
        int c0 = 0;
        hipError_t e = hipSuccess;
        while (e == hipSuccess && k - c0 >= 2 * CLv) {
            const int left = k - c0;
            if (left >= 8 * CLv) {
                e = launch(TypeBox<CoopSpmmSink<VT, 8>>(), 8 * CLv, c0);
                c0 += 8 * CLv;
            } else if (left >= 4 * CLv) {
                e = launch(TypeBox<CoopSpmmSink<VT, 4>>(), 4 * CLv, c0);
                c0 += 4 * CLv;
            } else {
                e = launch(TypeBox<CoopSpmmSink<VT, 2>>(), 2 * CLv, c0);
                c0 += 2 * CLv;
            }
        }
        if (e != hipSuccess || c0 == k) return e;
        X += c0;
        Y += c0;
        k -= c0;
    }
    // widest column chunk that fits the registers without spilling; FP32
    // accumulators only while a lane's sum has at most 32 terms, so that the
    // worst-case rounding error, (T - 1) 2^-24 |A||x|, stays below 2e-6 |A||x|
    const bool f32acc = std::is_same<VT, float>::value && a.layout == 2 && a.lane_nnz <= 32;
    const int kcmax = std::is_same<VT, double>::value ? 8 : 16;
    return for_kc(k, kcmax, [&](auto KCc, int c0) {
        constexpr int KC = decltype(KCc)::value;
        if constexpr (std::is_same<VT, float>::value && KC >= 8 && KC <= 16) {
            if (f32acc) return launch(TypeBox<SpmmSink<VT, KC, false, float>>(), KC, c0);
        }
        if constexpr (KC > 16 || (std::is_same<VT, double>::value && KC > 8)) {
            return hipErrorInvalidValue;  // excluded by kcmax
        } else {
            return launch(TypeBox<SpmmSink<VT, KC, false>>(), KC, c0);
        }
    });
}

// Columns of dX per pass of the LDS-privatised transpose (0: dX does not fit,
// use global atomics): the widest of 8, 4, 2, 1 whose n x KC block fits in
// LDS beside the tables, one 1024-thread workgroup per CU.
template <typename VT>
int trans_lds_cols(const DevMat &a) {
    const int64_t room = 160 * 1024 - 1024 - (int64_t)sizeof(Tables<VT>);
    for (int c : {8, 4, 2, 1})
        if ((a.n * c + a.n * c / 32 + 1) * (int64_t)sizeof(VT) <= room && a.n * c < (1ll << 31)) return c;
    return 0;
}

template <typename VT>
hipError_t spmm_t_impl(const DevMat &a, int k, const VT *dY, int64_t lddy, VT *dX, int64_t lddx,
                       double alpha, double beta, Launch L, void *work, size_t work_bytes,
                       hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    const int kcl = trans_lds_cols<VT>(a);
    const int64_t G = L.num_cus;
    if (kcl > 0 && a.nnz > 0 && a.num_waves > 0 &&
        work_bytes >= (size_t)G * (size_t)a.n * (size_t)kcl * sizeof(VT)) {
        VT *part = (VT *)work;
        return for_kc(k, kcl, [&](auto KCc, int c0) {
            constexpr int KC = decltype(KCc)::value;
            if constexpr (KC > 8) {
                return hipErrorInvalidValue;  // excluded by kcl
            } else {
                typename TransLdsSink<VT, KC>::Params sp;
                sp.dY = dY + c0;
                sp.lddy = (uint32_t)lddy;
                sp.lds = nullptr;
                const size_t dyn = ((size_t)a.n * KC + (size_t)a.n * KC / 32 + 1) * sizeof(VT);
                auto kern = a.layout == 1 ? pick_bd(a, trans_lds_kernel<1, VT, KC, 1>, trans_lds_kernel<1, VT, KC, 0>)
                                          : pick_bd(a, trans_lds_kernel<2, VT, KC, 1>, trans_lds_kernel<2, VT, KC, 0>);
                hipError_t e = hipFuncSetAttribute((const void *)kern,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL(kern, dim3((unsigned)G), dim3(1024), dyn, st, a, sp, part);
                e = hipGetLastError();
                if (e != hipSuccess) return e;
                const int64_t cnt = a.n * KC;
                hipLaunchKernelGGL(trans_reduce_kernel<VT>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                                   st, (const VT *)part, G, a.n, KC, dX + c0, lddx, alpha, beta);
                return hipGetLastError();
            }
        });
    }
    return for_kc(k, [&](auto KCc, int c0) {
        constexpr int KC = decltype(KCc)::value;
        const int64_t tot = a.n * KC;
        hipLaunchKernelGGL(scale_kernel<VT>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                           dX + c0, a.n, KC, lddx, beta);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || a.nnz == 0 || a.num_waves == 0) return e;
        typename TransSink<VT, KC>::Params sp;
        sp.dY = dY + c0;
        sp.lddy = (uint32_t)lddy;
        sp.dX = dX + c0;
        sp.lddx = (uint32_t)lddx;
        sp.alpha = alpha;
        typedef TransSink<VT, KC> TS;
        if (a.layout == 1)
            return launch_persistent(pick_bd(a, decode_kernel<1, VT, TS, TS::kOcc, 1>,
                                             decode_kernel<1, VT, TS, TS::kOcc, 0>),
                                     a, L, st, a, sp);
        return launch_persistent(pick_bd(a, decode_kernel<2, VT, TS, occ_nnz(TS::kOcc), 1>,
                                         decode_kernel<2, VT, TS, occ_nnz(TS::kOcc), 0>),
                                 a, L, st, a, sp);
    });
}

template <typename VT>
hipError_t decode_impl(const DevMat &a, int32_t *col, void *vals, Launch L, hipStream_t st) {
    if (a.nnz == 0 || a.num_waves == 0) return hipSuccess;
    typename DecodeSink<VT>::Params sp;
    sp.col = col;
    sp.vals = (typename Bits<VT>::T *)vals;
    typedef DecodeSink<VT> DS;
    if (a.layout == 1)
        return launch_persistent(pick_bd(a, decode_kernel<1, VT, DS, DS::kOcc, 1>, decode_kernel<1, VT, DS, DS::kOcc, 0>),
                                 a, L, st, a, sp);
    return launch_persistent(pick_bd(a, decode_kernel<2, VT, DS, occ_nnz(DS::kOcc), 1>,
                                     decode_kernel<2, VT, DS, occ_nnz(DS::kOcc), 0>),
                             a, L, st, a, sp);
}

template <typename VT>
hipError_t csr_impl(const CsrDev &c, int k, const VT *X, int64_t ldx, VT *Y, int64_t ldy,
                    double alpha, double beta, double *partial, int num_cus, hipStream_t st) {
    if (c.m == 0) return hipSuccess;
    return for_kc(k, [&](auto KCc, int c0) {
        constexpr int KC = decltype(KCc)::value;
        if (c.nnz == 0) {
            const int64_t tot = c.m * KC;
            hipLaunchKernelGGL(scale_kernel<VT>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                               st, Y + c0, c.m, KC, ldy, beta);
            return hipGetLastError();
        }
        if (c.variant == 3 && KC == 1 && ldx == 1 && ldy == 1) {
            hipLaunchKernelGGL(csr_stream_kernel<VT>, dim3((unsigned)c.nblk), dim3(256), 0, st, c,
                               c.blk, X + c0, Y + c0, alpha, beta);
            return hipGetLastError();
        }
        if (c.variant == 2) {
            hipLaunchKernelGGL((csr_split_kernel<VT, KC>), dim3((unsigned)((c.num_lanes + 255) / 256)),
                               dim3(256), 0, st, c, X + c0, ldx, Y + c0, ldy, alpha, beta, partial);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            return launch_fixup(c.split, partial, KC, 0, Y + c0, ldy, alpha, beta, st);
        }
        const int64_t rows_per_block = 256 / c.group;
        int64_t blocks = (c.m + rows_per_block - 1) / rows_per_block;
        blocks = blocks < (int64_t)num_cus * 8 ? blocks : (int64_t)num_cus * 8;
#define DTANS_CSR_G(GG)                                                                         \
    case GG:                                                                                    \
        hipLaunchKernelGGL((csr_vector_kernel<VT, GG, KC>), dim3((unsigned)blocks), dim3(256), 0, \
                           st, c, X + c0, ldx, Y + c0, ldy, alpha, beta);                      \
        break;
        switch (c.group) {
            DTANS_CSR_G(1)
            DTANS_CSR_G(2)
            DTANS_CSR_G(4)
            DTANS_CSR_G(8)
            DTANS_CSR_G(16)
            DTANS_CSR_G(32)
            DTANS_CSR_G(64)
            default:
                return hipErrorInvalidValue;
        }
#undef DTANS_CSR_G
        return hipGetLastError();
    });
}

}  // namespace

hipError_t launch_spmm(const DevMat &a, bool f64, int k, const void *X, int64_t ldx, void *Y,
                       int64_t ldy, double alpha, double beta, double *partial, Launch L,
                       hipStream_t st) {
    if (f64)
        return spmm_impl<double>(a, k, (const double *)X, ldx, (double *)Y, ldy, alpha, beta,
                                 partial, L, st);
    return spmm_impl<float>(a, k, (const float *)X, ldx, (float *)Y, ldy, alpha, beta, partial, L,
                            st);
}

size_t spmm_scratch_bytes(const DevMat &a, int k) {
    if (a.layout != 2 || a.nnz == 0) return 0;
    return (size_t)(2 * a.num_lanes * (int64_t)std::min(k, kMaxPassCols) + 1) * sizeof(double);
}

size_t spmm_t_work_bytes(const DevMat &a, bool f64, int num_cus) {
    const int c = f64 ? trans_lds_cols<double>(a) : trans_lds_cols<float>(a);
    return (size_t)num_cus * (size_t)a.n * (size_t)c * (f64 ? 8 : 4);
}

hipError_t launch_spmm_t(const DevMat &a, bool f64, int k, const void *dY, int64_t lddy, void *dX,
                         int64_t lddx, double alpha, double beta, Launch L, void *work,
                         size_t work_bytes, hipStream_t st) {
    if (f64)
        return spmm_t_impl<double>(a, k, (const double *)dY, lddy, (double *)dX, lddx, alpha, beta,
                                   L, work, work_bytes, st);
    return spmm_t_impl<float>(a, k, (const float *)dY, lddy, (float *)dX, lddx, alpha, beta, L,
                              work, work_bytes, st);
}

hipError_t launch_decode(const DevMat &a, bool f64, int32_t *col, void *vals, Launch L,
                         hipStream_t st) {
    return f64 ? decode_impl<double>(a, col, vals, L, st) : decode_impl<float>(a, col, vals, L, st);
}

// copies the x / y pointers of one call from the launch arguments into the
// batch's device pointer table (stream-ordered with the batch kernel)
__global__ void batch_ptrs_kernel(BatchPtrs p, int count, void **table) {
    const int i = threadIdx.x;
    if (i < count) {
        table[2 * i] = (void *)p.xs[i];
        table[2 * i + 1] = p.ys[i];
    }
}

hipError_t launch_batch(const BatchDev &b, const BatchPtrs &ptrs, int count, bool f64, double alpha,
                        double beta, Launch L, hipStream_t st) {
    hipLaunchKernelGGL(batch_ptrs_kernel, dim3(1), dim3(kMaxBatch), 0, st, ptrs, count,
                       (void **)b.ptrs);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
    const dim3 block(64 * L.waves_per_wg);
    if (f64)
        hipLaunchKernelGGL(batch_kernel<double>, dim3(L.grid), block, 0, st, b, alpha, beta);
    else
        hipLaunchKernelGGL(batch_kernel<float>, dim3(L.grid), block, 0, st, b, alpha, beta);
    return hipGetLastError();
}

template <typename VT>
hipError_t batch_spmm_impl(const BatchDev &b, int k, bool aligned, double alpha, double beta, Launch L,
                           hipStream_t st) {
    auto go = [&](auto kern, int c0) -> hipError_t {
        // the task lists hold for any workgroup size; the kernel may allow fewer
        // waves per workgroup than the plan (more registers per wave)
        hipFuncAttributes fa;
        int wpw = L.waves_per_wg;
        if (hipFuncGetAttributes(&fa, (const void *)kern) == hipSuccess)
            wpw = std::max(1, std::min(wpw, fa.maxThreadsPerBlock / 64));
        hipLaunchKernelGGL(kern, dim3(L.grid), dim3(64 * wpw), 0, st, b, c0, k, alpha, beta);
        return hipGetLastError();
    };
    constexpr int CL = 16 / (int)sizeof(VT);
    int c0 = 0;
    hipError_t e = hipSuccess;
    // lane groups sharing each row of X (16-byte pieces), then single columns
    while (aligned && e == hipSuccess && k - c0 >= 2 * CL) {
        if (k - c0 >= 8 * CL) {
            typedef CoopSpmmSink<VT, 8> S;
            e = go(batch_spmm_kernel<VT, S, S::kOcc>, c0);
            c0 += 8 * CL;
        } else if (k - c0 >= 4 * CL) {
            typedef CoopSpmmSink<VT, 4> S;
            e = go(batch_spmm_kernel<VT, S, S::kOcc>, c0);
            c0 += 4 * CL;
        } else {
            typedef CoopSpmmSink<VT, 2> S;
            e = go(batch_spmm_kernel<VT, S, S::kOcc>, c0);
            c0 += 2 * CL;
        }
    }
    while (e == hipSuccess && c0 < k) {
        if (k - c0 >= 4) {
            typedef SpmmSink<VT, 4, false> S;
            e = go(batch_spmm_kernel<VT, S, S::kOcc>, c0);
            c0 += 4;
        } else if (k - c0 >= 2) {
            typedef SpmmSink<VT, 2, false> S;
            e = go(batch_spmm_kernel<VT, S, S::kOcc>, c0);
            c0 += 2;
        } else {
            typedef SpmmSink<VT, 1, false> S;
            e = go(batch_spmm_kernel<VT, S, S::kOcc>, c0);
            c0 += 1;
        }
    }
    return e;
}

hipError_t launch_batch_spmm(const BatchDev &b, const BatchPtrs &ptrs, int count, bool f64, int k,
                             bool aligned, double alpha, double beta, Launch L, hipStream_t st) {
    hipLaunchKernelGGL(batch_ptrs_kernel, dim3(1), dim3(kMaxBatch), 0, st, ptrs, count,
                       (void **)b.ptrs);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
    return f64 ? batch_spmm_impl<double>(b, k, aligned, alpha, beta, L, st)
               : batch_spmm_impl<float>(b, k, aligned, alpha, beta, L, st);
}

hipError_t launch_flush(const void *buf, int64_t bytes, uint32_t *sink, hipStream_t st) {
    if (bytes % 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(flush_kernel, dim3(2048), dim3(256), 0, st, (const uint4 *)buf, bytes / 16, sink);
    return hipGetLastError();
}

hipError_t launch_csr(const CsrDev &c, bool f64, int k, const void *X, int64_t ldx, void *Y,
                      int64_t ldy, double alpha, double beta, double *partial, int num_cus,
                      hipStream_t st) {
    if (f64)
        return csr_impl<double>(c, k, (const double *)X, ldx, (double *)Y, ldy, alpha, beta, partial,
                                num_cus, st);
    return csr_impl<float>(c, k, (const float *)X, ldx, (float *)Y, ldy, alpha, beta, partial,
                           num_cus, st);
}

// Scratch for callers that cannot allocate device memory (dtans_spmm_noalloc):
// a file-scope array that every GPU the library runs on holds from the first
// use until the process ends.  On the host its name is only a stand-in
// symbol, so host code never passes it to a kernel, a memset or a copy: it
// looks up the device address of each GPU's own copy once, with that device
// current, and passes that address instead.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(void **ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace dtans
