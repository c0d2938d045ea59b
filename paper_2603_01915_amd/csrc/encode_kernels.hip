// The per-nonzero passes of the CSR-dtANS encoder on gfx950
// (DeviceEncoder): delta and value keys of every nonzero (Sec. IV-A), their
// histograms (radix sort + run-length encoding), the symbol of every nonzero
// (the host's hash map, probed the same way), and per wave the words (base
// pass, digit pass, Sec. IV-E, interleaved in the order the decoder's ballots
// consume them, Sec. IV-B) and the escape regions (Sec. IV-F).  The host
// validates the input, fits the alphabets and builds the tables between the
// two calls; the container is identical to the host encoder's.
//
// Words: one wavefront encodes one wave; lane q holds lane stream 64 w + q.
// enc_count_kernel runs every lane's base pass forward, keeps its load flags
// (2 bits per step) and sums the wave's word count; the host turns the counts
// into offsets; enc_words_kernel runs the digit pass backward from the wave's
// last step, placing each step's words at the end of what is left of the
// wave's region, and finally the three initial words of every lane.  Escapes
// take the same count / offsets / write scheme, forward.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <string>
#include <vector>

#include "container.hpp"
#include "dtans_core.hpp"

namespace dtans {
namespace {

struct WordJobDev {
    const int32_t *row_ptr;  // layout row: lane l holds row l
    const int32_t *dsym, *vsym;
    const uint32_t *dmeta, *vmeta;  // first | base << 16
    const uint16_t *dslots, *vslots;
    const uint64_t *flag_off;  // per wave, in 32-bit words; num_waves + 1
    uint32_t *flags;           // [wave][step / 16][lane], 2 bits per step
    uint64_t *wave_words;      // word count of every wave (first kernel)
    const uint64_t *word_off;  // num_waves + 1 (second kernel)
    uint32_t *words;
    int32_t *err;              // set when a wave's words do not fill its region
    int64_t nnz, num_lanes, num_waves;
    int32_t layout, lane_nnz, dpad, vpad;
};

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ uint32_t prefix_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// first nonzero and count of lane stream l (0 for lanes past the end)
__device__ __forceinline__ void lane_span(const WordJobDev &J, int64_t l, int64_t &g0, int64_t &cnt) {
    g0 = 0;
    cnt = 0;
    if (l >= J.num_lanes) return;
    if (J.layout == (int32_t)kLayoutRow) {
        g0 = J.row_ptr[l];
        cnt = (int64_t)J.row_ptr[l + 1] - g0;
    } else {
        g0 = l * (int64_t)J.lane_nnz;
        cnt = std::min<int64_t>(J.lane_nnz, J.nnz - g0);
    }
}

// the symbol of stream position t (even: a delta, odd: a value) and its
// alphabet's metadata; positions past the lane's nonzeros hold the padding
// symbols
__device__ __forceinline__ uint32_t meta_at(const WordJobDev &J, int64_t g0, int64_t cnt, int64_t t) {
    const int64_t i = t >> 1;
    if (t & 1) return J.vmeta[i < cnt ? J.vsym[g0 + i] : J.vpad];
    return J.dmeta[i < cnt ? J.dsym[g0 + i] : J.dpad];
}

__device__ __forceinline__ uint32_t slot_of(const WordJobDev &J, int64_t t, uint32_t meta, uint32_t digit) {
    const uint32_t at = (meta & 0xffffu) + digit;
    return (t & 1) ? J.vslots[at] : J.dslots[at];
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ int64_t wave_max(int64_t v) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) v = std::max<int64_t>(v, __shfl_xor(v, d, 64));
    return v;
}

// Base pass (Sec. IV-E): the radix r of the decoder's state after every digit
// group; a group whose product leaves r below 2^32 makes the decoder load a
// word.  Flags of step j: bit 2 (j mod 16) for group 1, the next bit for
// group 2.
__global__ __launch_bounds__(256) void enc_count_kernel(WordJobDev J) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= J.num_waves) return;  // whole wavefronts
    const uint32_t q = threadIdx.x & 63u;
    int64_t g0, cnt;
    lane_span(J, w * 64 + q, g0, cnt);
    const int64_t S = (cnt + 3) >> 2;
    uint32_t *fl = J.flags + J.flag_off[w] + q;
    uint64_t r = 1, loads = 0;
    uint32_t fw = 0;
    for (int64_t j = 0; j + 1 < S; ++j) {
        for (int g = 0; g < 2; ++g) {
            for (int k = 0; k < 4; ++k) r *= (meta_at(J, g0, cnt, 8 * j + 4 * g + k) >> 16);
            if (r >> 32) {
                r >>= 32;
            } else {
                fw |= 1u << (2 * (j & 15) + g);
                ++loads;
            }
        }
        if ((j & 15) == 15 || j + 2 == S) {
            fl[(j >> 4) * 64] = fw;
            fw = 0;
        }
    }
    const uint64_t mine = S > 0 ? 3 + (uint64_t)(S - 1) + loads : 0;
    const uint64_t total = wave_sum(mine);
    if (q == 0) J.wave_words[w] = total;
}

// Digit pass (Sec. IV-E), backward from state 0 with the last segment's
// digits 0: the words read at step j are the packed slots of segment j + 1;
// after writing them, the state takes each group's word (unless that group
// loads it, Sec. IV-D) and gives up one digit per symbol, last symbol first.
__global__ __launch_bounds__(256) void enc_words_kernel(WordJobDev J) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= J.num_waves) return;
    const uint32_t q = threadIdx.x & 63u;
    int64_t g0, cnt;
    lane_span(J, w * 64 + q, g0, cnt);
    const int64_t S = (cnt + 3) >> 2;
    const int64_t maxS = wave_max(S);
    const uint32_t *fl = J.flags + J.flag_off[w] + q;
    uint32_t slots[8];
    if (S > 0) {
        for (int k = 0; k < 8; ++k) {
            const int64_t t = 8 * (S - 1) + k;
            slots[k] = slot_of(J, t, meta_at(J, g0, cnt, t), 0);
        }
    } else {
        for (int k = 0; k < 8; ++k) slots[k] = 0;
    }
    uint64_t d = 0;
    const uint64_t ms = wave_ballot(S > 0);
    const uint32_t live = (uint32_t)__popcll(ms);
    // the words of the steps fill [word_off[w] + 3 live, word_off[w + 1]);
    // a count that disagrees with the first kernel's stops the wave before
    // it writes outside its region
    const uint64_t floor = J.word_off[w] + 3ull * live;
    uint64_t pos = J.word_off[w + 1];
    for (int64_t j = maxS - 2; j >= 0; --j) {
        const bool act = j + 1 < S;
        uint32_t nw[3];
        pack8(slots, nw[0], nw[1], nw[2]);
        const uint32_t fw = act ? fl[(j >> 4) * 64] >> (2 * (j & 15)) : 0u;
        const bool f1 = act && (fw & 1u), f2 = act && (fw & 2u);
        const uint64_t m1 = wave_ballot(f1), m2 = wave_ballot(f2), m3 = wave_ballot(act);
        const uint32_t c1 = (uint32_t)__popcll(m1), c2 = (uint32_t)__popcll(m2);
        const uint32_t step_words = c1 + c2 + (uint32_t)__popcll(m3);
        if (pos < floor + step_words) {  // uniform
            if (q == 0) atomicOr(J.err, 1);
            return;
        }
        pos -= step_words;
        if (f1) J.words[pos + prefix_below(m1)] = nw[0];
        if (f2) J.words[pos + c1 + prefix_below(m2)] = nw[1];
        if (act) J.words[pos + c1 + c2 + prefix_below(m3)] = nw[2];
        if (act) {
            for (int g = 1; g >= 0; --g) {
                const bool loaded = g ? f2 : f1;
                if (!loaded) d = (d << 32) | nw[g];
                for (int k = 4 * g + 3; k >= 4 * g; --k) {
                    const int64_t t = 8 * j + k;
                    const uint32_t meta = meta_at(J, g0, cnt, t);
                    const uint32_t b = meta >> 16;
                    const uint32_t dig = (uint32_t)(d % b);
                    d /= b;
                    slots[k] = slot_of(J, t, meta, dig);
                }
            }
        }
    }
    if (pos != floor) {
        if (q == 0) atomicOr(J.err, 1);
        return;
    }
    if (S > 0) {
        uint32_t iw[3];
        pack8(slots, iw[0], iw[1], iw[2]);
        for (int k = 0; k < 3; ++k) J.words[J.word_off[w] + (uint64_t)k * live + prefix_below(ms)] = iw[k];
    }
}

// Delta key of every nonzero g (Sec. IV-A): the difference to the previous
// column, except at the start of a row or of a lane stream, where it is the
// column relative to first_base of the row holding g.  The row is found by a
// binary search of row_ptr (the last i with row_ptr[i] <= g).  Columns out of
// [0, n) or below their predecessor in the row are reported in *bad as the
// smallest 2 g + (1 for unsorted), the error a serial scan finds first.
__global__ __launch_bounds__(256) void enc_keys_kernel(const int32_t *__restrict__ row_ptr, int64_t m,
                                                       const int32_t *__restrict__ col, int64_t nnz, int64_t n,
                                                       int32_t layout, int32_t lane_nnz, uint32_t first_mode,
                                                       uint32_t *__restrict__ dkey,
                                                       unsigned long long *__restrict__ bad) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < nnz;
         g += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = m;  // row_ptr[lo] <= g < row_ptr[hi]
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (row_ptr[mid] <= g) lo = mid;
            else hi = mid;
        }
        const bool row_start = row_ptr[lo] == g;
        const bool lane_start = layout == (int32_t)kLayoutRow ? row_start : g % lane_nnz == 0;
        const int32_t cg = col[g];
        const uint32_t c = (uint32_t)cg;
        dkey[g] = (row_start || lane_start) ? c - first_base(first_mode, (uint32_t)lo)
                                            : c - (uint32_t)col[g - 1];
        if (cg < 0 || cg >= n) atomicMin(bad, (unsigned long long)(2 * g));
        else if (!row_start && cg < col[g - 1]) atomicMin(bad, (unsigned long long)(2 * g + 1));
    }
}

struct DevAlphabet {
    const uint64_t *hkey;
    const int32_t *hval;
    uint64_t mask;
    int32_t esc;
};

__device__ __forceinline__ int32_t lookup(const DevAlphabet &a, uint64_t key) {
    uint64_t h = ((key * 0x9e3779b97f4a7c15ull) >> 40) & a.mask;
    while (a.hval[h] >= 0) {  // the map always has empty entries
        if (a.hkey[h] == key) return a.hval[h];
        h = (h + 1) & a.mask;
    }
    return a.esc;
}

template <typename VK>
__global__ __launch_bounds__(256) void enc_lookup_kernel(const uint32_t *__restrict__ dkey,
                                                         const VK *__restrict__ vkey, int64_t nnz,
                                                         DevAlphabet da, DevAlphabet va,
                                                         int32_t *__restrict__ dsym, int32_t *__restrict__ vsym) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < nnz;
         g += (int64_t)gridDim.x * blockDim.x) {
        dsym[g] = lookup(da, dkey[g]);
        vsym[g] = lookup(va, (uint64_t)vkey[g]);
    }
}

// escaped deltas and values of every wave (counts, then the regions in the
// decoder's order: segment j, its nonzero k, then lane)
struct EscJob {
    const int32_t *row_ptr;
    const int32_t *dsym, *vsym;
    const uint32_t *dkey;
    const void *vals;
    int32_t desc, vesc, f64;
    int64_t nnz, num_lanes, num_waves;
    int32_t layout, lane_nnz;
    uint64_t *dcount, *vcount;           // per wave (count kernel)
    const uint64_t *doff, *voff;         // num_waves + 1 (write kernel)
    uint32_t *escd;
    uint64_t *escv;
    int32_t *err;
};

__device__ __forceinline__ void esc_span(const EscJob &J, int64_t l, int64_t &g0, int64_t &cnt) {
    g0 = 0;
    cnt = 0;
    if (l >= J.num_lanes) return;
    if (J.layout == (int32_t)kLayoutRow) {
        g0 = J.row_ptr[l];
        cnt = (int64_t)J.row_ptr[l + 1] - g0;
    } else {
        g0 = l * (int64_t)J.lane_nnz;
        cnt = std::min<int64_t>(J.lane_nnz, J.nnz - g0);
    }
}

__global__ __launch_bounds__(256) void enc_esc_count_kernel(EscJob J) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= J.num_waves) return;
    const uint32_t q = threadIdx.x & 63u;
    int64_t g0, cnt;
    esc_span(J, w * 64 + q, g0, cnt);
    uint64_t nd = 0, nv = 0;
    for (int64_t i = 0; i < cnt; ++i) {
        nd += J.dsym[g0 + i] == J.desc;
        nv += J.vsym[g0 + i] == J.vesc;
    }
    nd = wave_sum(nd);
    nv = wave_sum(nv);
    if (q == 0) {
        J.dcount[w] = nd;
        J.vcount[w] = nv;
    }
}

__global__ __launch_bounds__(256) void enc_esc_write_kernel(EscJob J) {
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= J.num_waves) return;
    const uint32_t q = threadIdx.x & 63u;
    int64_t g0, cnt;
    esc_span(J, w * 64 + q, g0, cnt);
    const int64_t maxS = wave_max((cnt + 3) >> 2);
    uint64_t pd = J.doff[w], pv = J.voff[w];
    const uint64_t ed = J.doff[w + 1], ev = J.voff[w + 1];
    for (int64_t t = 0; t < 4 * maxS; ++t) {  // t = 4 j + k
        const bool live = t < cnt;
        const bool fd = live && J.dsym[g0 + t] == J.desc;
        const bool fv = live && J.vsym[g0 + t] == J.vesc;
        const uint64_t md = wave_ballot(fd), mv = wave_ballot(fv);
        const uint64_t nd = (uint64_t)__popcll(md), nv = (uint64_t)__popcll(mv);
        if (pd + nd > ed || pv + nv > ev) {  // uniform; never expected
            if (q == 0) atomicOr(J.err, 1);
            return;
        }
        if (fd) J.escd[pd + prefix_below(md)] = J.dkey[g0 + t];
        if (fv)
            J.escv[pv + prefix_below(mv)] = J.f64 ? ((const uint64_t *)J.vals)[g0 + t]
                                                  : (uint64_t)((const uint32_t *)J.vals)[g0 + t];
        pd += nd;
        pv += nv;
    }
}

// device buffers of one encoder, freed with it
struct DevBuffers {
    std::vector<void *> ptrs;
    ~DevBuffers() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    hipError_t alloc(T *&p, size_t count) {
        void *v = nullptr;
        hipError_t e = hipMalloc(&v, std::max<size_t>(1, count) * sizeof(T));
        if (e != hipSuccess) return e;
        ptrs.push_back(v);
        p = (T *)v;
        return hipSuccess;
    }
};

std::string hip_fail(hipError_t e, const char *what) {
    return std::string(e == hipErrorOutOfMemory ? "ENOMEM: " : "EHIP: ") + what + ": " + hipGetErrorString(e);
}

#define ENC_TRY(call)                                     \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

unsigned elem_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

// sorted (key, count) pairs of n keys of type K on the device
template <typename K>
std::string device_histogram(const K *keys, int64_t n, hipStream_t st, std::vector<KeyCount> &out) {
    out.clear();
    if (n == 0) return "";
    DevBuffers B;
    K *sorted = nullptr, *uniq = nullptr;
    int32_t *counts = nullptr, *runs = nullptr;
    ENC_TRY(B.alloc(sorted, n));
    ENC_TRY(B.alloc(uniq, n));
    ENC_TRY(B.alloc(counts, n));
    ENC_TRY(B.alloc(runs, 1));
    size_t a = 0, b = 0;
    ENC_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, a, keys, sorted, (int)n, 0, (int)(8 * sizeof(K)), st));
    ENC_TRY(hipcub::DeviceRunLengthEncode::Encode(nullptr, b, sorted, uniq, counts, runs, (int)n, st));
    uint8_t *tmp = nullptr;
    ENC_TRY(B.alloc(tmp, std::max(a, b)));
    size_t ta = std::max(a, b), tb = ta;
    ENC_TRY(hipcub::DeviceRadixSort::SortKeys(tmp, ta, keys, sorted, (int)n, 0, (int)(8 * sizeof(K)), st));
    ENC_TRY(hipcub::DeviceRunLengthEncode::Encode(tmp, tb, sorted, uniq, counts, runs, (int)n, st));
    int32_t nr = 0;
    ENC_TRY(hipMemcpyAsync(&nr, runs, 4, hipMemcpyDeviceToHost, st));
    ENC_TRY(hipStreamSynchronize(st));
    if (nr < 0 || nr > n) return "ECORRUPT: device histogram";
    std::vector<K> hk(nr);
    std::vector<int32_t> hc(nr);
    if (nr) {
        ENC_TRY(hipMemcpyAsync(hk.data(), uniq, nr * sizeof(K), hipMemcpyDeviceToHost, st));
        ENC_TRY(hipMemcpyAsync(hc.data(), counts, nr * 4, hipMemcpyDeviceToHost, st));
        ENC_TRY(hipStreamSynchronize(st));
    }
    out.resize(nr);
    for (int32_t i = 0; i < nr; ++i) out[i] = {(uint64_t)hk[i], (int64_t)hc[i]};
    return "";
}

class GpuEncoder final : public DeviceEncoder {
  public:
    GpuEncoder(void *stream, bool device_inputs) : st_((hipStream_t)stream), dev_in_(device_inputs) {}

    bool inputs_on_device() const override { return dev_in_; }

    std::string keys(const Container &c, const int32_t *col, const void *vals, std::vector<KeyCount> &dhist,
                     std::vector<KeyCount> &vhist) override {
        const int64_t nnz = c.nnz;
        f64_ = c.dtype == kF64;
        const size_t vb = f64_ ? 8 : 4;
        unsigned long long *bad = nullptr;
        ENC_TRY(B_.alloc(rp_, c.row_ptr.size()));
        ENC_TRY(B_.alloc(dkey_, nnz));
        ENC_TRY(B_.alloc(bad, 1));
        if (dev_in_) {
            col_ = (int32_t *)col;
            vals_ = (uint8_t *)vals;
        } else {
            ENC_TRY(B_.alloc(col_, nnz));
            ENC_TRY(B_.alloc(vals_, nnz * vb));
        }
        ENC_TRY(hipMemcpyAsync(rp_, c.row_ptr.data(), c.row_ptr.size() * 4, hipMemcpyHostToDevice, st_));
        ENC_TRY(hipMemsetAsync(bad, 0xff, 8, st_));
        if (nnz) {
            if (!dev_in_) {
                ENC_TRY(hipMemcpyAsync(col_, col, nnz * 4, hipMemcpyHostToDevice, st_));
                ENC_TRY(hipMemcpyAsync(vals_, vals, nnz * vb, hipMemcpyHostToDevice, st_));
            }
            hipLaunchKernelGGL(enc_keys_kernel, dim3(elem_grid(nnz)), dim3(256), 0, st_, rp_, c.m, col_, nnz, c.n,
                               (int32_t)c.layout, (int32_t)c.lane_nnz, c.first_mode, dkey_, bad);
            ENC_TRY(hipGetLastError());
        }
        unsigned long long hbad = 0;
        ENC_TRY(hipMemcpyAsync(&hbad, bad, 8, hipMemcpyDeviceToHost, st_));
        ENC_TRY(hipStreamSynchronize(st_));
        if (hbad != ~0ull) {
            const int64_t g = (int64_t)(hbad >> 1), row = row_of(c.row_ptr, g);
            if (hbad & 1) return "EUNSORTED: columns not ascending in row " + std::to_string(row);
            return "ERANGE: column index out of range in row " + std::to_string(row);
        }
        std::string e = device_histogram(dkey_, nnz, st_, dhist);
        if (!e.empty()) return e;
        if (f64_) return device_histogram((const uint64_t *)vals_, nnz, st_, vhist);
        return device_histogram((const uint32_t *)vals_, nnz, st_, vhist);
    }

    std::string streams(const AlphabetMap &da, const AlphabetMap &va, Container &c) override;

  private:
    hipStream_t st_;
    bool dev_in_;
    DevBuffers B_;
    bool f64_ = false;
    int32_t *rp_ = nullptr, *col_ = nullptr;
    uint8_t *vals_ = nullptr;
    uint32_t *dkey_ = nullptr;
};

std::string GpuEncoder::streams(const AlphabetMap &da, const AlphabetMap &va, Container &c) {
    const int64_t W = c.num_waves, nnz = c.nnz;
    c.words.clear();
    c.escd.clear();
    c.escv.clear();
    c.word_off.assign(W + 1, 0);
    c.escd_off.assign(W + 1, 0);
    c.escv_off.assign(W + 1, 0);
    if (W == 0) return "";
    auto in_range = [](int32_t s, size_t n) { return s >= 0 && (size_t)s < n; };
    if (nnz > 0 && (!in_range(da.pad, da.meta.size()) || !in_range(va.pad, va.meta.size())))
        return "EUNSUPPORTED: an alphabet without a padding symbol";
    for (const AlphabetMap *a : {&da, &va}) {
        const size_t h = a->hkey.size();
        if (h == 0 || (h & (h - 1)) || a->hval.size() != h) return "ECORRUPT: bad symbol map";
    }
    // flag words per wave: 64 lanes x ceil(steps / 16), steps = maxS - 1
    std::vector<uint64_t> flag_off(W + 1, 0);
    for (int64_t w = 0; w < W; ++w) {
        int64_t maxS = 0;
        for (int q = 0; q < 64; ++q) {
            const int64_t l = w * 64 + q;
            if (l >= c.num_lanes) break;
            int64_t g0, cnt;
            c.lane_range(l, g0, cnt);
            maxS = std::max(maxS, (cnt + 3) / 4);
        }
        const int64_t steps = maxS > 0 ? maxS - 1 : 0;
        flag_off[w + 1] = flag_off[w] + 64 * (uint64_t)((steps + 15) / 16);
    }
    DevBuffers B;
    int32_t *ds = nullptr, *vs = nullptr, *err = nullptr, *dhv = nullptr, *vhv = nullptr;
    uint32_t *dm = nullptr, *vm = nullptr, *fl = nullptr, *wd = nullptr, *escd = nullptr;
    uint16_t *dsl = nullptr, *vsl = nullptr;
    uint64_t *fo = nullptr, *ww = nullptr, *wo = nullptr, *dhk = nullptr, *vhk = nullptr;
    uint64_t *dc = nullptr, *vc = nullptr, *doff = nullptr, *voff = nullptr, *escv = nullptr;
    ENC_TRY(B.alloc(ds, nnz));
    ENC_TRY(B.alloc(vs, nnz));
    ENC_TRY(B.alloc(dhk, da.hkey.size()));
    ENC_TRY(B.alloc(vhk, va.hkey.size()));
    ENC_TRY(B.alloc(dhv, da.hval.size()));
    ENC_TRY(B.alloc(vhv, va.hval.size()));
    ENC_TRY(B.alloc(dm, da.meta.size()));
    ENC_TRY(B.alloc(vm, va.meta.size()));
    ENC_TRY(B.alloc(dsl, da.slots.size()));
    ENC_TRY(B.alloc(vsl, va.slots.size()));
    ENC_TRY(B.alloc(fo, W + 1));
    ENC_TRY(B.alloc(fl, flag_off[W]));
    ENC_TRY(B.alloc(ww, W));
    ENC_TRY(B.alloc(wo, W + 1));
    ENC_TRY(B.alloc(dc, W));
    ENC_TRY(B.alloc(vc, W));
    ENC_TRY(B.alloc(doff, W + 1));
    ENC_TRY(B.alloc(voff, W + 1));
    ENC_TRY(B.alloc(err, 1));
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st_) : hipSuccess;
    };
    ENC_TRY(up(dhk, da.hkey.data(), da.hkey.size() * 8));
    ENC_TRY(up(vhk, va.hkey.data(), va.hkey.size() * 8));
    ENC_TRY(up(dhv, da.hval.data(), da.hval.size() * 4));
    ENC_TRY(up(vhv, va.hval.data(), va.hval.size() * 4));
    ENC_TRY(up(dm, da.meta.data(), da.meta.size() * 4));
    ENC_TRY(up(vm, va.meta.data(), va.meta.size() * 4));
    ENC_TRY(up(dsl, da.slots.data(), da.slots.size() * 2));
    ENC_TRY(up(vsl, va.slots.data(), va.slots.size() * 2));
    ENC_TRY(up(fo, flag_off.data(), (W + 1) * 8));
    ENC_TRY(hipMemsetAsync(err, 0, 4, st_));
    // symbols
    if (nnz) {
        const DevAlphabet dA = {dhk, dhv, da.hkey.size() - 1, da.esc}, vA = {vhk, vhv, va.hkey.size() - 1, va.esc};
        if (f64_)
            hipLaunchKernelGGL(enc_lookup_kernel<uint64_t>, dim3(elem_grid(nnz)), dim3(256), 0, st_, dkey_,
                               (const uint64_t *)vals_, nnz, dA, vA, ds, vs);
        else
            hipLaunchKernelGGL(enc_lookup_kernel<uint32_t>, dim3(elem_grid(nnz)), dim3(256), 0, st_, dkey_,
                               (const uint32_t *)vals_, nnz, dA, vA, ds, vs);
        ENC_TRY(hipGetLastError());
    }
    // counts of words and escapes per wave
    WordJobDev J = {};
    J.row_ptr = rp_;
    J.dsym = ds;
    J.vsym = vs;
    J.dmeta = dm;
    J.vmeta = vm;
    J.dslots = dsl;
    J.vslots = vsl;
    J.flag_off = fo;
    J.flags = fl;
    J.wave_words = ww;
    J.word_off = wo;
    J.words = nullptr;
    J.err = err;
    J.nnz = nnz;
    J.num_lanes = c.num_lanes;
    J.num_waves = W;
    J.layout = (int32_t)c.layout;
    J.lane_nnz = (int32_t)c.lane_nnz;
    J.dpad = da.pad;
    J.vpad = va.pad;
    EscJob E = {};
    E.row_ptr = rp_;
    E.dsym = ds;
    E.vsym = vs;
    E.dkey = dkey_;
    E.vals = vals_;
    E.desc = da.esc;
    E.vesc = va.esc;
    E.f64 = f64_ ? 1 : 0;
    E.nnz = nnz;
    E.num_lanes = c.num_lanes;
    E.num_waves = W;
    E.layout = (int32_t)c.layout;
    E.lane_nnz = (int32_t)c.lane_nnz;
    E.dcount = dc;
    E.vcount = vc;
    E.doff = doff;
    E.voff = voff;
    E.err = err;
    const dim3 grid((unsigned)((W + 3) / 4)), block(256);
    hipLaunchKernelGGL(enc_count_kernel, grid, block, 0, st_, J);
    ENC_TRY(hipGetLastError());
    hipLaunchKernelGGL(enc_esc_count_kernel, grid, block, 0, st_, E);
    ENC_TRY(hipGetLastError());
    std::vector<uint64_t> cw(W), cd(W), cv(W);
    ENC_TRY(hipMemcpyAsync(cw.data(), ww, W * 8, hipMemcpyDeviceToHost, st_));
    ENC_TRY(hipMemcpyAsync(cd.data(), dc, W * 8, hipMemcpyDeviceToHost, st_));
    ENC_TRY(hipMemcpyAsync(cv.data(), vc, W * 8, hipMemcpyDeviceToHost, st_));
    ENC_TRY(hipStreamSynchronize(st_));
    for (int64_t w = 0; w < W; ++w) {
        c.word_off[w + 1] = c.word_off[w] + cw[w];
        c.escd_off[w + 1] = c.escd_off[w] + cd[w];
        c.escv_off[w + 1] = c.escv_off[w] + cv[w];
    }
    ENC_TRY(B.alloc(wd, c.word_off[W]));
    ENC_TRY(B.alloc(escd, c.escd_off[W]));
    ENC_TRY(B.alloc(escv, c.escv_off[W]));
    J.words = wd;
    E.escd = escd;
    E.escv = escv;
    ENC_TRY(up(wo, c.word_off.data(), (W + 1) * 8));
    ENC_TRY(up(doff, c.escd_off.data(), (W + 1) * 8));
    ENC_TRY(up(voff, c.escv_off.data(), (W + 1) * 8));
    hipLaunchKernelGGL(enc_words_kernel, grid, block, 0, st_, J);
    ENC_TRY(hipGetLastError());
    if (c.escd_off[W] + c.escv_off[W]) {
        hipLaunchKernelGGL(enc_esc_write_kernel, grid, block, 0, st_, E);
        ENC_TRY(hipGetLastError());
    }
    c.words.resize(c.word_off[W]);
    c.escd.resize(c.escd_off[W]);
    c.escv.resize(c.escv_off[W]);
    auto down = [&](void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st_) : hipSuccess;
    };
    int32_t herr = 0;
    ENC_TRY(down(c.words.data(), wd, c.words.size() * 4));
    ENC_TRY(down(c.escd.data(), escd, c.escd.size() * 4));
    ENC_TRY(down(c.escv.data(), escv, c.escv.size() * 8));
    ENC_TRY(down(&herr, err, 4));
    ENC_TRY(hipStreamSynchronize(st_));
    if (herr) return "ECORRUPT: device encoder: a wave's words or escapes do not fill its region";
    return "";
}

}  // namespace

DeviceEncoder *new_device_encoder(void *stream, bool device_inputs) { return new GpuEncoder(stream, device_inputs); }

}  // namespace dtans
