// Device word pass of the CSR-dtANS encoder for gfx950: for every lane
// stream the base pass (which steps load a word after each digit group) and
// the digit pass (the slots of every segment and the words they pack into,
// Sec. IV-E), and the interleave of the 64 lane streams of a wave in the
// order the decoder's ballots consume them (Sec. IV-B).  The host fits the
// alphabets, builds the tables, maps every nonzero to its two symbols and
// writes the escape regions; this pass produces the words and the per-wave
// word offsets, identical to the host encoder's.
//
// One wavefront encodes one wave; lane q holds lane stream 64 w + q.  Two
// kernels: the first runs every lane's base pass forward, keeps its load
// flags (2 bits per step) and sums the wave's word count; the host turns the
// counts into offsets; the second runs the digit pass backward from the
// wave's last step, placing each step's words at the end of what is left of
// the wave's region, and finally the three initial words of every lane.
#include <hip/hip_runtime.h>

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

// device buffers of one coder call, freed on every path
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

}  // namespace

#define ENC_TRY(call)                                  \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// WordCoder on the current device; ctx is the hipStream_t to run on.
std::string device_word_coder(const WordJob &job, void *ctx, std::vector<uint32_t> &words,
                              std::vector<uint64_t> &word_off) {
    const Container &c = *job.c;
    hipStream_t st = (hipStream_t)ctx;
    const int64_t W = c.num_waves;
    words.clear();
    word_off.assign(W + 1, 0);
    if (W == 0) return "";
    auto in_range = [](int32_t s, size_t n) { return s >= 0 && (size_t)s < n; };
    if (c.nnz > 0 && (!in_range(job.dpad, job.dmeta.size()) || !in_range(job.vpad, job.vmeta.size())))
        return "EUNSUPPORTED: an alphabet without a padding symbol";
    // flag words per wave: 64 lanes x ceil((steps) / 16), steps = maxS - 1
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
    const size_t nnz = (size_t)c.nnz;
    DevBuffers B;
    WordJobDev J = {};
    int32_t *rp = nullptr, *ds = nullptr, *vs = nullptr, *err = nullptr;
    uint32_t *dm = nullptr, *vm = nullptr, *fl = nullptr, *wd = nullptr;
    uint16_t *dsl = nullptr, *vsl = nullptr;
    uint64_t *fo = nullptr, *ww = nullptr, *wo = nullptr;
    const bool row = c.layout == kLayoutRow;
    ENC_TRY(B.alloc(rp, row ? c.row_ptr.size() : 1));
    ENC_TRY(B.alloc(ds, nnz));
    ENC_TRY(B.alloc(vs, nnz));
    ENC_TRY(B.alloc(dm, job.dmeta.size()));
    ENC_TRY(B.alloc(vm, job.vmeta.size()));
    ENC_TRY(B.alloc(dsl, job.dslots.size()));
    ENC_TRY(B.alloc(vsl, job.vslots.size()));
    ENC_TRY(B.alloc(fo, W + 1));
    ENC_TRY(B.alloc(fl, flag_off[W]));
    ENC_TRY(B.alloc(ww, W));
    ENC_TRY(B.alloc(wo, W + 1));
    ENC_TRY(B.alloc(err, 1));
    if (row) ENC_TRY(hipMemcpyAsync(rp, c.row_ptr.data(), c.row_ptr.size() * 4, hipMemcpyHostToDevice, st));
    if (nnz) {
        ENC_TRY(hipMemcpyAsync(ds, job.dsym, nnz * 4, hipMemcpyHostToDevice, st));
        ENC_TRY(hipMemcpyAsync(vs, job.vsym, nnz * 4, hipMemcpyHostToDevice, st));
    }
    ENC_TRY(hipMemcpyAsync(dm, job.dmeta.data(), job.dmeta.size() * 4, hipMemcpyHostToDevice, st));
    ENC_TRY(hipMemcpyAsync(vm, job.vmeta.data(), job.vmeta.size() * 4, hipMemcpyHostToDevice, st));
    ENC_TRY(hipMemcpyAsync(dsl, job.dslots.data(), job.dslots.size() * 2, hipMemcpyHostToDevice, st));
    ENC_TRY(hipMemcpyAsync(vsl, job.vslots.data(), job.vslots.size() * 2, hipMemcpyHostToDevice, st));
    ENC_TRY(hipMemcpyAsync(fo, flag_off.data(), (W + 1) * 8, hipMemcpyHostToDevice, st));
    ENC_TRY(hipMemsetAsync(err, 0, 4, st));
    J.row_ptr = rp;
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
    J.nnz = c.nnz;
    J.num_lanes = c.num_lanes;
    J.num_waves = W;
    J.layout = (int32_t)c.layout;
    J.lane_nnz = (int32_t)c.lane_nnz;
    J.dpad = job.dpad;
    J.vpad = job.vpad;
    const dim3 grid((unsigned)((W + 3) / 4)), block(256);
    hipLaunchKernelGGL(enc_count_kernel, grid, block, 0, st, J);
    ENC_TRY(hipGetLastError());
    std::vector<uint64_t> counts(W);
    ENC_TRY(hipMemcpyAsync(counts.data(), ww, W * 8, hipMemcpyDeviceToHost, st));
    ENC_TRY(hipStreamSynchronize(st));
    for (int64_t w = 0; w < W; ++w) word_off[w + 1] = word_off[w] + counts[w];
    ENC_TRY(B.alloc(wd, word_off[W]));
    J.words = wd;
    ENC_TRY(hipMemcpyAsync(wo, word_off.data(), (W + 1) * 8, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(enc_words_kernel, grid, block, 0, st, J);
    ENC_TRY(hipGetLastError());
    words.resize(word_off[W]);
    int32_t herr = 0;
    if (word_off[W]) ENC_TRY(hipMemcpyAsync(words.data(), wd, word_off[W] * 4, hipMemcpyDeviceToHost, st));
    ENC_TRY(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st));
    ENC_TRY(hipStreamSynchronize(st));
    if (herr) return "ECORRUPT: device word pass: a wave's words do not fill its region";
    return "";
}

}  // namespace dtans
