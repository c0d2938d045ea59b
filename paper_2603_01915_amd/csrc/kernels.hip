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

#include <type_traits>

#include "dtans_core.hpp"
#include "kernels.hpp"

namespace dtans {
namespace {

constexpr int kComplete = 0, kHead = 1, kTail = 2;
constexpr int kNumXcd = 8;

__device__ __forceinline__ uint32_t lane_prefix(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    return v;
}

// workgroup index renumbered so that consecutive numbers share an XCD
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t G) {
    const int64_t x = b % kNumXcd, p = b / kNumXcd;
    const int64_t q = G / kNumXcd, r = G % kNumXcd;
    return x * q + (x < r ? x : r) + p;
}

template <typename VT> struct Bits;
template <> struct Bits<double> { typedef uint64_t T; };
template <> struct Bits<float> { typedef uint32_t T; };

template <typename VT>
__device__ __forceinline__ VT load_value(const void *p, uint64_t i) {
    return ((const VT *)p)[i];
}

// ------------------------------------------------------------------ sinks
// A sink consumes the decoded nonzeros of one lane in order:
//   nz(g, row, col, v): nonzero number g (row-major), its row, column, value
//   row_done(row, kind): the lane has seen its last nonzero of `row`; kind
//     says whether the lane holds the whole row, its head (the row started in
//     an earlier lane) or its tail (the row continues in later lanes).

template <typename VT, int KC>
struct SpmmSink {
    struct Params {
        const VT *X;
        int64_t ldx;
        VT *Y;
        int64_t ldy;
        double *partial;  // [lane][head/tail][KC]
        int64_t n;
        double alpha, beta;
    };
    const Params p;
    int64_t lane;
    double acc[KC];
    __device__ SpmmSink(const Params &pp, int64_t l) : p(pp), lane(l) {
#pragma unroll
        for (int c = 0; c < KC; ++c) acc[c] = 0.0;
    }
    __device__ __forceinline__ void nz(int64_t, int32_t, uint32_t col, VT v) {
        const uint32_t cc = min(col, (uint32_t)(p.n - 1));  // memory safety only
        const VT *x = p.X + (int64_t)cc * p.ldx;
#pragma unroll
        for (int c = 0; c < KC; ++c) acc[c] = fma((double)v, (double)x[c], acc[c]);
    }
    __device__ __forceinline__ void row_done(int32_t row, int kind) {
        if (kind == kComplete) {
            VT *y = p.Y + (int64_t)row * p.ldy;
#pragma unroll
            for (int c = 0; c < KC; ++c)
                y[c] = (VT)(p.beta == 0.0 ? p.alpha * acc[c] : p.alpha * acc[c] + p.beta * (double)y[c]);
        } else {
            double *q = p.partial + (2 * lane + (kind == kTail ? 1 : 0)) * KC;
#pragma unroll
            for (int c = 0; c < KC; ++c) q[c] = acc[c];
        }
#pragma unroll
        for (int c = 0; c < KC; ++c) acc[c] = 0.0;
    }
};

template <typename VT, int KC>
struct TransSink {
    struct Params {
        const VT *dY;
        int64_t lddy;
        VT *dX;
        int64_t lddx;
        int64_t n;
        double alpha;
    };
    const Params p;
    int32_t cur = -1;
    VT dy[KC];
    __device__ TransSink(const Params &pp, int64_t) : p(pp) {}
    __device__ __forceinline__ void nz(int64_t, int32_t row, uint32_t col, VT v) {
        if (row != cur) {
            cur = row;
            const VT *src = p.dY + (int64_t)row * p.lddy;
#pragma unroll
            for (int c = 0; c < KC; ++c) dy[c] = (VT)(p.alpha * (double)src[c]);
        }
        const uint32_t cc = min(col, (uint32_t)(p.n - 1));
        VT *dst = p.dX + (int64_t)cc * p.lddx;
#pragma unroll
        for (int c = 0; c < KC; ++c) unsafeAtomicAdd(dst + c, v * dy[c]);
    }
    __device__ __forceinline__ void row_done(int32_t, int) {}
};

template <typename VT>
struct DecodeSink {
    struct Params {
        int32_t *col;
        typename Bits<VT>::T *vals;
    };
    const Params p;
    __device__ DecodeSink(const Params &pp, int64_t) : p(pp) {}
    __device__ __forceinline__ void nz(int64_t g, int32_t, uint32_t col, VT v) {
        p.col[g] = (int32_t)col;
        p.vals[g] = __builtin_bit_cast(typename Bits<VT>::T, v);
    }
    __device__ __forceinline__ void row_done(int32_t, int) {}
};

// --------------------------------------------------------- wave decoding
// Decode encoded wave `slice` (lanes slice*64 .. slice*64+63) and feed the
// nonzeros of this thread's lane to `sink`.
template <int LAYOUT, typename VT, class Sink>
__device__ __forceinline__ void decode_slice(const DevMat &a, const uint64_t *__restrict__ tab,
                                             const VT *__restrict__ tval, int64_t slice,
                                             uint32_t lane, Sink &sink) {
    const int64_t l = slice * kWave + lane;
    const bool live = l < a.num_lanes;
    int64_t g0 = 0, cnt = 0;
    int32_t row = 0, row_beg = 0, row_end = 0;
    if (live) {
        if (LAYOUT == 1) {
            row = (int32_t)l;
            row_beg = a.row_ptr[l];
            cnt = a.row_ptr[l + 1] - row_beg;
            g0 = row_beg;
        } else {
            g0 = l * (int64_t)a.lane_nnz;
            cnt = min((int64_t)a.lane_nnz, a.nnz - g0);
            row = a.lane_row[l];
            row_beg = a.row_ptr[row];
            row_end = a.row_ptr[row + 1];
        }
    }
    const int S = (int)((cnt + 3) >> 2);
    const int Smax = wave_max(S);

    // per-wave stream bases are uniform; offsets into them stay 32-bit and
    // uniform (popcounts of ballots), so the compiler keeps them in SGPRs
    const uint32_t *__restrict__ W = a.words + a.woff[slice];
    const uint32_t *__restrict__ ED = a.escd + a.doff[slice];
    const VT *__restrict__ EV = (const VT *)a.escv + a.voff[slice];
    uint32_t pos, dpos = 0, vpos = 0;
    uint32_t w1, w2, w3;
    {
        // lanes without a stream read a neighbouring word (buffers are padded)
        const uint64_t mk = __ballot(S > 0);
        const uint32_t pre = lane_prefix(mk), c = (uint32_t)__popcll(mk);
        w1 = W[pre];
        w2 = W[c + pre];
        w3 = W[2 * c + pre];
        pos = 3 * c;
    }
    uint32_t d = 0, r = 1, col = 0;
    int64_t g = g0;
    for (int j = 0; j < Smax; ++j) {
        const bool act = j < S;
        const bool more = j + 1 < S;
        const int rem = (int)cnt - 4 * j;
        uint32_t sl[8];
        unpack8(w1, w2, w3, sl);
        uint64_t e[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) e[k] = tab[sl[k]];
        VT v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = tval[sl[2 * k + 1]];
        // The next segment's words first, so that their loads are in flight
        // while this segment's escapes and x gathers are served.  Loads are
        // issued by every lane and the extracted word selected afterwards;
        // lanes that do not load read a neighbouring word of the stream.
        if (j + 1 < Smax) {
            uint32_t D, Rm1, x1, x2;
            group4((uint32_t)(e[0] >> 32) & 0xffffu, (uint32_t)(e[1] >> 48),
                   (uint32_t)(e[2] >> 32) & 0xffffu, (uint32_t)(e[3] >> 48), D, Rm1);
            const bool ext1 = append_and_check(d, r, D, Rm1, x1);
            group4((uint32_t)(e[4] >> 32) & 0xffffu, (uint32_t)(e[5] >> 48),
                   (uint32_t)(e[6] >> 32) & 0xffffu, (uint32_t)(e[7] >> 48), D, Rm1);
            const bool ext2 = append_and_check(d, r, D, Rm1, x2);
            const uint64_t m1 = __ballot(more && !ext1);
            const uint64_t m2 = __ballot(more && !ext2);
            const uint64_t m3 = __ballot(more);
            const uint32_t c1 = (uint32_t)__popcll(m1), c2 = (uint32_t)__popcll(m2);
            const uint32_t l1 = W[pos + lane_prefix(m1)];
            const uint32_t l2 = W[pos + c1 + lane_prefix(m2)];
            const uint32_t l3 = W[pos + c1 + c2 + lane_prefix(m3)];
            pos += c1 + c2 + (uint32_t)__popcll(m3);
            w1 = ext1 ? x1 : l1;
            w2 = ext2 ? x2 : l2;
            w3 = l3;
        }
        uint32_t dl[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) dl[k] = (uint32_t)e[2 * k] & (kDeltaLimit - 1);
        // escape flags: bit 31 of a delta slot's word, bit 30 of a value
        // slot's word.  Padding symbols are never escapes, so only lanes past
        // their last segment need masking.
        const uint32_t escd_any = (uint32_t)e[0] | (uint32_t)e[2] | (uint32_t)e[4] | (uint32_t)e[6];
        const uint32_t escv_any = (uint32_t)e[1] | (uint32_t)e[3] | (uint32_t)e[5] | (uint32_t)e[7];
        if (__ballot(act && (((escd_any >> 1) | escv_any) & (1u << 30)))) {  // wave-uniform
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool f = act && k < rem && ((uint32_t)e[2 * k] >> 31);
                const uint64_t mk = __ballot(f);
                if (f) dl[k] = ED[dpos + lane_prefix(mk)];
                dpos += (uint32_t)__popcll(mk);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool f = act && k < rem && (((uint32_t)e[2 * k + 1] >> 30) & 1u);
                const uint64_t mk = __ballot(f);
                if (f) v[k] = EV[vpos + lane_prefix(mk)];
                vpos += (uint32_t)__popcll(mk);
            }
        }
        if (LAYOUT == 1) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                col += dl[k];
                if (act && k < rem) sink.nz(g + k, row, col, v[k]);
            }
            g += 4;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (act && k < rem) {
                    while (g >= row_end) {  // rows ending before this nonzero
                        sink.row_done(row, row_beg < g0 ? kHead : kComplete);
                        col = 0;
                        ++row;
                        row_beg = row_end;
                        row_end = a.row_ptr[row + 1];
                    }
                    col += dl[k];
                    sink.nz(g, row, col, v[k]);
                    ++g;
                }
            }
        }
    }
    if (!live) return;
    if (LAYOUT == 1) {
        if (l < a.m) sink.row_done(row, kComplete);
    } else {
        const int64_t gend = g0 + cnt;
        while (row < a.m && row_end <= gend) {  // rows finished here, incl. empty ones
            sink.row_done(row, row_beg < g0 ? kHead : kComplete);
            ++row;
            row_beg = row_end;
            if (row < a.m) row_end = a.row_ptr[row + 1];
        }
        if (row < a.m && row_beg < gend) sink.row_done(row, row_beg < g0 ? kHead : kTail);
    }
}

template <typename VT>
__device__ __forceinline__ void stage_tables(const DevMat &a, uint64_t *s_tab, VT *s_val) {
    const VT *tv = (const VT *)a.tabval;
    for (int i = threadIdx.x; i < kSlots; i += blockDim.x) {
        s_tab[i] = a.tab[i];
        s_val[i] = tv[i];
    }
    __syncthreads();
}

// MINW: waves per SIMD the register allocation must allow (8 lets two
// 16-wave workgroups share a CU, which is what the LDS tables permit)
template <int LAYOUT, typename VT, class Sink, int MINW>
__global__ __launch_bounds__(1024, MINW) void decode_kernel(DevMat a, typename Sink::Params sp) {
    __shared__ uint64_t s_tab[kSlots];
    __shared__ VT s_val[kSlots];
    stage_tables<VT>(a, s_tab, s_val);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const int64_t wpb = blockDim.x / kWave;
    const int64_t total = (int64_t)gridDim.x * wpb;
    // the wave index is uniform; readfirstlane lets the compiler know it
    const int64_t gw = xcd_block(blockIdx.x, gridDim.x) * wpb +
                       __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t s0 = gw * a.num_waves / total, s1 = (gw + 1) * a.num_waves / total;
    for (int64_t s = s0; s < s1; ++s) {
        Sink sink(sp, s * kWave + lane);
        decode_slice<LAYOUT, VT>(a, s_tab, s_val, s, lane, sink);
    }
}

// rows split over lanes (layout NNZ): y = alpha * (tail of the first lane +
// heads of the following lanes) + beta * y
template <typename VT>
__global__ void fixup_kernel(const int32_t *split_row, const int32_t *first, const int32_t *last,
                             int64_t nsplit, const double *partial, int KC, VT *Y, int64_t ldy,
                             double alpha, double beta) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsplit * KC) return;
    const int64_t s = i / KC, c = i % KC;
    const int64_t a = first[s], b = last[s];
    double sum = partial[(2 * a + 1) * KC + c];
    for (int64_t l = a + 1; l <= b; ++l) sum += partial[(2 * l) * KC + c];
    VT *y = Y + (int64_t)split_row[s] * ldy + c;
    *y = (VT)(beta == 0.0 ? alpha * sum : alpha * sum + beta * (double)*y);
}

// Y[rows, :KC] = beta * Y (beta == 0: zero)
template <typename VT>
__global__ void scale_kernel(VT *Y, int64_t rows, int KC, int64_t ldy, double beta) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * KC) return;
    VT *y = Y + (i / KC) * ldy + i % KC;
    *y = beta == 0.0 ? (VT)0 : (VT)(beta * (double)*y);
}

// ------------------------------------------------- multi-matrix launch
template <typename VT>
__global__ __launch_bounds__(1024, 7) void batch_kernel(BatchDev b, double alpha, double beta) {
    __shared__ uint64_t s_tab[kSlots];
    __shared__ VT s_val[kSlots];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), wpb = blockDim.x / kWave;
    const int t0 = b.wg_task[blockIdx.x], t1 = b.wg_task[blockIdx.x + 1];
    int cur = -1;
    for (int t = t0; t < t1; ++t) {
        const BatchTask task = b.tasks[t];
        const DevMat &a = b.mats[task.mat];
        if (task.mat != cur) {  // restage the tables only when the matrix changes
            __syncthreads();
            const VT *tv = (const VT *)a.tabval;
            for (int i = threadIdx.x; i < kSlots; i += blockDim.x) {
                s_tab[i] = a.tab[i];
                s_val[i] = tv[i];
            }
            __syncthreads();
            cur = task.mat;
        }
        typename SpmmSink<VT, 1>::Params sp;
        sp.X = (const VT *)b.xs[task.mat];
        sp.ldx = 1;
        sp.Y = (VT *)b.ys[task.mat];
        sp.ldy = 1;
        sp.partial = nullptr;
        sp.n = a.n;
        sp.alpha = alpha;
        sp.beta = beta;
        for (int w = wib; w < task.num_waves; w += wpb) {
            const int64_t s = task.first_wave + w;
            SpmmSink<VT, 1> sink(sp, s * kWave + lane);
            decode_slice<1, VT>(a, s_tab, s_val, s, lane, sink);
        }
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

// ------------------------------------------------------------ dispatch
template <typename F>
hipError_t for_kc(int k, F f) {
    // split k columns into compile-time chunks
    int c0 = 0;
    while (c0 < k) {
        int left = k - c0;
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

template <typename VT>
hipError_t spmm_impl(const DevMat &a, int k, const VT *X, int64_t ldx, VT *Y, int64_t ldy,
                     double alpha, double beta, double *partial, Launch L, hipStream_t st) {
    const dim3 block(64 * L.waves_per_wg);
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
    return for_kc(k, [&](auto KCc, int c0) {
        constexpr int KC = decltype(KCc)::value;
        typename SpmmSink<VT, KC>::Params sp;
        sp.X = X + c0;
        sp.ldx = ldx;
        sp.Y = Y + c0;
        sp.ldy = ldy;
        sp.partial = partial;
        sp.n = a.n;
        sp.alpha = alpha;
        sp.beta = beta;
        if (a.layout == 1)
            hipLaunchKernelGGL((decode_kernel<1, VT, SpmmSink<VT, KC>, (KC <= 2 ? 7 : 4)>), dim3(L.grid), block, 0, st,
                               a, sp);
        else
            hipLaunchKernelGGL((decode_kernel<2, VT, SpmmSink<VT, KC>, (KC <= 2 ? 7 : 4)>), dim3(L.grid), block, 0, st,
                               a, sp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (a.layout == 2 && a.nsplit > 0) {
            const int64_t tot = a.nsplit * KC;
            hipLaunchKernelGGL(fixup_kernel<VT>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                               st, a.split_row, a.split_first, a.split_last, a.nsplit, partial, KC,
                               Y + c0, ldy, alpha, beta);
            e = hipGetLastError();
        }
        return e;
    });
}

template <typename VT>
hipError_t spmm_t_impl(const DevMat &a, int k, const VT *dY, int64_t lddy, VT *dX, int64_t lddx,
                       double alpha, double beta, Launch L, hipStream_t st) {
    if (a.n == 0) return hipSuccess;
    return for_kc(k, [&](auto KCc, int c0) {
        constexpr int KC = decltype(KCc)::value;
        const int64_t tot = a.n * KC;
        hipLaunchKernelGGL(scale_kernel<VT>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                           dX + c0, a.n, KC, lddx, beta);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || a.nnz == 0 || a.num_waves == 0) return e;
        typename TransSink<VT, KC>::Params sp;
        sp.dY = dY + c0;
        sp.lddy = lddy;
        sp.dX = dX + c0;
        sp.lddx = lddx;
        sp.n = a.n;
        sp.alpha = alpha;
        const dim3 block(64 * L.waves_per_wg);
        if (a.layout == 1)
            hipLaunchKernelGGL((decode_kernel<1, VT, TransSink<VT, KC>, (KC <= 2 ? 7 : 4)>), dim3(L.grid), block, 0,
                               st, a, sp);
        else
            hipLaunchKernelGGL((decode_kernel<2, VT, TransSink<VT, KC>, (KC <= 2 ? 7 : 4)>), dim3(L.grid), block, 0,
                               st, a, sp);
        return hipGetLastError();
    });
}

template <typename VT>
hipError_t decode_impl(const DevMat &a, int32_t *col, void *vals, Launch L, hipStream_t st) {
    if (a.nnz == 0 || a.num_waves == 0) return hipSuccess;
    typename DecodeSink<VT>::Params sp;
    sp.col = col;
    sp.vals = (typename Bits<VT>::T *)vals;
    const dim3 block(64 * L.waves_per_wg);
    if (a.layout == 1)
        hipLaunchKernelGGL((decode_kernel<1, VT, DecodeSink<VT>, 7>), dim3(L.grid), block, 0, st, a, sp);
    else
        hipLaunchKernelGGL((decode_kernel<2, VT, DecodeSink<VT>, 7>), dim3(L.grid), block, 0, st, a, sp);
    return hipGetLastError();
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
        if (c.variant == 2) {
            hipLaunchKernelGGL((csr_split_kernel<VT, KC>), dim3((unsigned)((c.num_lanes + 255) / 256)),
                               dim3(256), 0, st, c, X + c0, ldx, Y + c0, ldy, alpha, beta, partial);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess || c.nsplit == 0) return e;
            const int64_t tot = c.nsplit * KC;
            hipLaunchKernelGGL(fixup_kernel<VT>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                               st, c.split_row, c.split_first, c.split_last, c.nsplit, partial, KC,
                               Y + c0, ldy, alpha, beta);
            return hipGetLastError();
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

hipError_t launch_spmm_t(const DevMat &a, bool f64, int k, const void *dY, int64_t lddy, void *dX,
                         int64_t lddx, double alpha, double beta, Launch L, hipStream_t st) {
    if (f64)
        return spmm_t_impl<double>(a, k, (const double *)dY, lddy, (double *)dX, lddx, alpha, beta,
                                   L, st);
    return spmm_t_impl<float>(a, k, (const float *)dY, lddy, (float *)dX, lddx, alpha, beta, L,
                              st);
}

hipError_t launch_decode(const DevMat &a, bool f64, int32_t *col, void *vals, Launch L,
                         hipStream_t st) {
    return f64 ? decode_impl<double>(a, col, vals, L, st) : decode_impl<float>(a, col, vals, L, st);
}

hipError_t launch_batch(const BatchDev &b, bool f64, double alpha, double beta, Launch L,
                        hipStream_t st) {
    const dim3 block(64 * L.waves_per_wg);
    if (f64)
        hipLaunchKernelGGL(batch_kernel<double>, dim3(L.grid), block, 0, st, b, alpha, beta);
    else
        hipLaunchKernelGGL(batch_kernel<float>, dim3(L.grid), block, 0, st, b, alpha, beta);
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

}  // namespace dtans
