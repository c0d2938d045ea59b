// Host-side CSR-dtANS encoder, container I/O and verifying decoder.
//
// Encoding follows Sec. IV of Schaetzle, Pegolotti, Pueschel, "Fast Entropy
// Decoding for Sparse MVM on GPUs" (2026):
//  * column indices are delta-encoded per row; the first delta of a row (and,
//    in the nonzero-balanced layout, of a lane stream) is the column itself
//    (Sec. IV-A) or, in first-delta mode 1 (this library's default, not the
//    paper's), the column relative to the row (dtans_core.hpp, kFirstBias);
//  * every nonzero contributes a delta symbol followed by a value symbol; the
//    lane streams of a 64-lane wave are interleaved word by word in the order
//    the decoder's ballots consume them (Sec. IV-B);
//  * each alphabet is fitted to K = 4096 slots with multiplicities at most
//    M = 256 (by default at most 255, see EncodeParams) plus an escape symbol whose raw payload goes to a separate
//    region, minimising the expected size (Sec. IV-C, IV-F);
//  * a forward base pass fixes the decoder's branches and a backward digit
//    pass chooses slots and emits words (Sec. IV-E);
//  * rows are padded to whole segments and the last segment of a lane stream
//    loads nothing (Sec. IV-F); slots are randomly permuted (Sec. IV-F).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <fstream>
#include <queue>
#include <thread>
#include <unordered_map>

#include "container.hpp"

namespace dtans {
namespace {

std::string fail(const char *cls, const std::string &msg) { return std::string(cls) + ": " + msg; }

int thread_count(int req) {
    if (req > 0) return req;
    unsigned h = std::thread::hardware_concurrency();
    return h ? (int)std::min(h, 32u) : 4;
}

template <class F>
void parallel_chunks(int64_t n, int threads, F f) {
    if (n <= 0) return;
    threads = (int)std::min<int64_t>(threads, n);
    if (threads <= 1) {
        f(0, n, 0);
        return;
    }
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t) {
        int64_t b = n * t / threads, e = n * (t + 1) / threads;
        pool.emplace_back([=, &f] { f(b, e, t); });
    }
    for (auto &th : pool) th.join();
}

uint64_t splitmix_next(uint64_t &state) {
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

uint64_t fnv1a(const uint8_t *p, size_t n, uint64_t h = 0xcbf29ce484222325ull) {
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

// --------------------------------------------------------------- histograms
std::vector<KeyCount> histogram(const std::vector<uint64_t> &keys, int threads) {
    const int64_t n = (int64_t)keys.size();
    int T = (int)std::max<int64_t>(1, std::min<int64_t>(threads, n / 65536 + 1));
    std::vector<std::vector<KeyCount>> part(T);
    parallel_chunks(n, T, [&](int64_t b, int64_t e, int t) {
        std::vector<uint64_t> tmp(keys.begin() + b, keys.begin() + e);
        std::sort(tmp.begin(), tmp.end());
        auto &out = part[t];
        for (size_t i = 0; i < tmp.size();) {
            size_t j = i;
            while (j < tmp.size() && tmp[j] == tmp[i]) ++j;
            out.push_back({tmp[i], (int64_t)(j - i)});
            i = j;
        }
    });
    // pairwise merge of the sorted runs
    while (part.size() > 1) {
        std::vector<std::vector<KeyCount>> next;
        for (size_t i = 0; i + 1 < part.size(); i += 2) {
            std::vector<KeyCount> m;
            m.reserve(part[i].size() + part[i + 1].size());
            size_t a = 0, b = 0;
            auto &A = part[i], &B = part[i + 1];
            while (a < A.size() || b < B.size()) {
                if (b == B.size() || (a < A.size() && A[a].key < B[b].key)) m.push_back(A[a++]);
                else if (a == A.size() || B[b].key < A[a].key) m.push_back(B[b++]);
                else { m.push_back({A[a].key, A[a].count + B[b].count}); ++a; ++b; }
            }
            next.push_back(std::move(m));
        }
        if (part.size() % 2) next.push_back(std::move(part.back()));
        part.swap(next);
    }
    return part.empty() ? std::vector<KeyCount>() : std::move(part[0]);
}

// ------------------------------------------------------------ table fitting
// Multiplicities maximising sum c_i log m_i subject to sum m_i <= K and
// 1 <= m_i <= cap (cap <= M): greedy increments by marginal gain (optimal for this
// separable concave objective).  Returns the coded bits sum c_i log2(K/m_i).
double allocate(const std::vector<int64_t> &c, std::vector<int> &mult, int cap) {
    const size_t q = c.size();
    mult.assign(q, 1);
    int left = kSlots - (int)q;
    typedef std::pair<double, int> Gain;
    std::priority_queue<Gain> heap;
    for (size_t i = 0; i < q; ++i)
        if (c[i] > 0) heap.push({(double)c[i] * log2(2.0), (int)i});
    while (left > 0 && !heap.empty()) {
        Gain g = heap.top();
        heap.pop();
        int i = g.second;
        mult[i]++;
        --left;
        if (mult[i] < cap)
            heap.push({(double)c[i] * log2((mult[i] + 1.0) / mult[i]), i});
    }
    double bits = 0;
    for (size_t i = 0; i < q; ++i)
        if (c[i] > 0) bits += (double)c[i] * log2((double)kSlots / mult[i]);
    return bits;
}

struct Fit {
    std::vector<uint64_t> keys;  // table symbols, in allocation order
    std::vector<int64_t> counts;
    std::vector<int> mult;
    bool escape = false;
    int esc_mult = 0;
    int64_t esc_count = 0;
};

// Choose which symbols get table slots and their multiplicities so that the
// expected encoded size (coded bits + raw bits of escaped symbols) is
// smallest over a search of the table size.
Fit fit_alphabet(const std::vector<KeyCount> &hist, int raw_bits, bool is_delta, int cap, int threads) {
    std::vector<KeyCount> cand;
    int64_t forced_esc = 0;
    for (const auto &kc : hist) {
        if (is_delta && kc.key >= kDeltaLimit) forced_esc += kc.count;
        else cand.push_back(kc);
    }
    std::sort(cand.begin(), cand.end(), [](const KeyCount &a, const KeyCount &b) {
        return a.count != b.count ? a.count > b.count : a.key < b.key;
    });
    Fit best;
    int64_t total = forced_esc;
    for (const auto &kc : cand) total += kc.count;
    if (total == 0) return best;
    if (cand.empty()) {  // keep one ordinary symbol so that padding has one
        cand.push_back({0, 0});
    }
    std::vector<int64_t> suffix(cand.size() + 1, 0);
    for (size_t i = cand.size(); i-- > 0;) suffix[i] = suffix[i + 1] + cand[i].count;
    const int tmax = (int)std::min<size_t>(cand.size(), kSlots);
    auto evaluate = [&](int t, Fit *out) -> double {
        int64_t esc = forced_esc + suffix[t];
        if (esc > 0 && t > kSlots - 1) return INFINITY;
        std::vector<int64_t> c(t);
        for (int i = 0; i < t; ++i) c[i] = cand[i].count;
        if (esc > 0) c.push_back(esc);
        std::vector<int> mult;
        double bits = allocate(c, mult, cap) + (double)esc * raw_bits;
        if (out) {
            out->keys.resize(t);
            out->counts.resize(t);
            for (int i = 0; i < t; ++i) {
                out->keys[i] = cand[i].key;
                out->counts[i] = cand[i].count;
            }
            out->mult.assign(mult.begin(), mult.begin() + t);
            out->escape = esc > 0;
            out->esc_mult = esc > 0 ? mult[t] : 0;
            out->esc_count = esc;
        }
        return bits;
    };
    // Every table size is evaluated (the size is not unimodal in t, so a
    // coarse search can miss the optimum; for a fixed t the t most frequent
    // admissible keys are an optimal choice, since an escaped symbol costs
    // more than its raw bits >= 32 while a table slot costs at most
    // log2(K) = 12 bits).  The sizes are evaluated in parallel, then scanned
    // in order: the first strictly smaller size wins.
    std::vector<double> bits(tmax);
    // sizes dealt round-robin: an evaluation costs more for small t
    const int nth = std::max(1, std::min(threads, tmax));
    parallel_chunks((int64_t)nth, nth, [&](int64_t b, int64_t e, int) {
        for (int64_t w = b; w < e; ++w)
            for (int t = (int)w + 1; t <= tmax; t += nth) bits[t - 1] = evaluate(t, nullptr);
    });
    double best_bits = INFINITY;
    int best_t = 1;
    for (int t = 1; t <= tmax; ++t)
        if (bits[t - 1] < best_bits) { best_bits = bits[t - 1]; best_t = t; }
    evaluate(best_t, &best);
    return best;
}

// Slot assignment: symbols take consecutive logical slots (digits 0..m-1),
// the escape last, then a seeded Fisher-Yates permutation spreads them over
// the physical slots (Sec. IV-F).
struct SlotMap {
    std::vector<uint64_t> keys;       // symbol index -> key
    std::vector<int> mult;            // symbol index -> base
    std::vector<int> first;           // symbol index -> offset into slots
    std::vector<uint16_t> slots;      // flat: slots of symbol s by digit
    int esc_index = -1;
    // open-addressing key -> symbol index
    std::vector<uint64_t> hkey;
    std::vector<int32_t> hval;
    int lookup(uint64_t key) const {
        size_t mask = hkey.size() - 1;
        size_t h = (size_t)((key * 0x9e3779b97f4a7c15ull) >> 40) & mask;
        while (hval[h] >= 0) {
            if (hkey[h] == key) return hval[h];
            h = (h + 1) & mask;
        }
        return esc_index;
    }
};

void build_table(const Fit &fit, uint64_t seed, Table &tab, SlotMap &sm) {
    tab = Table();
    sm = SlotMap();
    const int t = (int)fit.keys.size();
    const int nsym = t + (fit.escape ? 1 : 0);
    sm.keys = fit.keys;
    sm.mult = fit.mult;
    if (fit.escape) {
        sm.keys.push_back(0);
        sm.mult.push_back(fit.esc_mult);
        sm.esc_index = t;
    }
    std::vector<uint16_t> perm(kSlots);
    for (int i = 0; i < kSlots; ++i) perm[i] = (uint16_t)i;
    uint64_t st = seed;
    for (int i = kSlots - 1; i > 0; --i) {
        int j = (int)(splitmix_next(st) % (uint64_t)(i + 1));
        std::swap(perm[i], perm[j]);
    }
    int logical = 0;
    sm.first.resize(nsym);
    for (int s = 0; s < nsym; ++s) {
        sm.first[s] = logical;
        for (int dgt = 0; dgt < sm.mult[s]; ++dgt) {
            uint16_t slot = perm[logical++];
            sm.slots.push_back(slot);
            tab.sym[slot] = (s == sm.esc_index) ? 0 : sm.keys[s];
            tab.digit[slot] = (uint8_t)dgt;
            tab.base[slot] = (uint16_t)sm.mult[s];
            tab.flags[slot] = (uint8_t)(1 | (s == sm.esc_index ? 2 : 0));
        }
    }
    tab.symbols = t;
    tab.has_escape = fit.escape;
    size_t hsize = 16;
    while (hsize < 4 * (size_t)std::max(t, 1)) hsize <<= 1;
    sm.hkey.assign(hsize, 0);
    sm.hval.assign(hsize, -1);
    for (int s = 0; s < t; ++s) {
        size_t mask = hsize - 1;
        size_t h = (size_t)((sm.keys[s] * 0x9e3779b97f4a7c15ull) >> 40) & mask;
        while (sm.hval[h] >= 0) h = (h + 1) & mask;
        sm.hkey[h] = sm.keys[s];
        sm.hval[h] = s;
    }
}

// padding symbol: the one on the lowest-numbered used non-escape slot
int pad_symbol(const Table &tab, const SlotMap &sm) {
    for (int i = 0; i < kSlots; ++i)
        if ((tab.flags[i] & 1) && !(tab.flags[i] & 2)) return sm.lookup(tab.sym[i]);
    return -1;
}

void table_stats(const Fit &fit, int64_t total, Table &tab) {
    if (total == 0) return;
    double h = 0, hc = 0;
    for (size_t i = 0; i < fit.keys.size(); ++i) {
        if (!fit.counts[i]) continue;
        double p = (double)fit.counts[i] / total;
        h -= p * log2(p);
        hc += p * log2((double)kSlots / fit.mult[i]);
    }
    if (fit.escape && fit.esc_count) {
        double p = (double)fit.esc_count / total;
        hc += p * log2((double)kSlots / fit.esc_mult);
    }
    tab.entropy = h;  // over the table symbols (escaped ones are counted separately)
    tab.cross_entropy = hc;
}

// ----------------------------------------------------------- lane encoding
struct LaneCode {
    int64_t S = 0;
    uint32_t init[3] = {0, 0, 0};
    std::vector<uint8_t> load;   // 2 per step: conditional load after group 1 / 2
    std::vector<uint32_t> w;     // 3 per step: words for the next segment
};

struct Alpha {
    const SlotMap *sm;
};

// sym: 8*S symbol indices (delta, value alternating), padded
void encode_lane(const int32_t *sym, int64_t S, const SlotMap &dsm, const SlotMap &vsm,
                 LaneCode &L) {
    L.S = S;
    if (S == 0) return;
    const int64_t steps = S - 1;
    L.load.assign(2 * steps, 0);
    L.w.assign(3 * steps, 0);
    auto base = [&](int64_t t) -> uint64_t {
        return (uint64_t)((t & 1) ? vsm.mult[sym[t]] : dsm.mult[sym[t]]);
    };
    // base pass: radix only (Sec. IV-E)
    uint64_t r = 1;
    for (int64_t j = 0; j < steps; ++j)
        for (int g = 0; g < 2; ++g) {
            for (int k = 0; k < 4; ++k) r *= base(8 * j + 4 * g + k);
            if (r >> 32) r >>= 32;
            else L.load[2 * j + g] = 1;
        }
    // digit pass: backwards from state 0, last segment's digits 0
    uint32_t slots[8];
    for (int k = 0; k < 8; ++k) {
        int64_t t = 8 * (S - 1) + k;
        const SlotMap &sm = (k & 1) ? vsm : dsm;
        slots[k] = sm.slots[sm.first[sym[t]]];
    }
    uint64_t d = 0;
    for (int64_t j = steps - 1; j >= 0; --j) {
        uint32_t nw[3];
        pack8(slots, nw[0], nw[1], nw[2]);
        L.w[3 * j] = nw[0];
        L.w[3 * j + 1] = nw[1];
        L.w[3 * j + 2] = nw[2];
        for (int g = 1; g >= 0; --g) {
            if (!L.load[2 * j + g]) d = (d << 32) | nw[g];
            for (int k = 4 * g + 3; k >= 4 * g; --k) {
                int64_t t = 8 * j + k;
                const SlotMap &sm = (k & 1) ? vsm : dsm;
                uint64_t b = (uint64_t)sm.mult[sym[t]];
                uint64_t dig = d % b;
                d /= b;
                slots[k] = sm.slots[sm.first[sym[t]] + dig];
            }
        }
    }
    pack8(slots, L.init[0], L.init[1], L.init[2]);
}

struct WaveOut {
    std::vector<uint32_t> words, escd;
    std::vector<uint64_t> escv;
    std::vector<uint64_t> woff, doff, voff;  // per wave, relative to this chunk
    std::string error;
};

}  // namespace

// ---------------------------------------------------------------- encode
std::string encode_csr(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                       const int32_t *col, const void *vals, uint32_t dtype,
                       const EncodeParams &p, Container &c, DeviceEncoder *dev) {
    if (m < 0 || n < 0 || nnz < 0) return fail("EINVAL", "negative size");
    if (m >= (1ll << 31) || n >= (1ll << 31) || nnz >= (1ll << 31))
        return fail("ERANGE", "rows, columns and nonzeros must be below 2^31");
    if (dtype != kF32 && dtype != kF64) return fail("EINVAL", "dtype must be F32 or F64");
    if (p.layout != kLayoutRow && p.layout != kLayoutNnz) return fail("EINVAL", "bad layout");
    if (p.layout == kLayoutNnz && (p.lane_nnz == 0 || p.lane_nnz % 4 != 0 || p.lane_nnz > (1u << 24)))
        return fail("EINVAL", "lane_nnz must be a positive multiple of 4");
    if (p.esc_mode > 1) return fail("EINVAL", "escape mode must be 0 (separate) or 1 (in stream)");
    if (!row_ptr || (nnz > 0 && (!col || !vals))) return fail("EINVAL", "null array");
    if (row_ptr[0] != 0 || row_ptr[m] != nnz) return fail("EINVAL", "row_ptr must run from 0 to nnz");
    if (p.sigma) {
        // sorted rows: encode the row-permuted matrix, keep the order
        if (p.layout != kLayoutRow || p.sigma % kWave)
            return fail("EINVAL", "a row-sort window needs the ROW layout and a multiple of 64 rows");
        if (dev && dev->inputs_on_device())
            return fail("EUNSUPPORTED", "rows of device-resident arrays are encoded in CSR order");
        for (int64_t i = 0; i < m; ++i)
            if (row_ptr[i + 1] < row_ptr[i]) return fail("EINVAL", "row_ptr decreases at row " + std::to_string(i));
        std::vector<int32_t> perm, rp2(m + 1), c2(nnz);
        sigma_order(m, row_ptr, p.sigma, perm);
        const size_t vb = dtype == kF64 ? 8 : 4;
        std::vector<uint8_t> v2(vb * (size_t)nnz);
        rp2[0] = 0;
        for (int64_t r = 0; r < m; ++r) {
            const int32_t i = perm[r], len = row_ptr[i + 1] - row_ptr[i];
            std::copy(col + row_ptr[i], col + row_ptr[i] + len, c2.begin() + rp2[r]);
            memcpy(&v2[vb * (size_t)rp2[r]], (const uint8_t *)vals + vb * (size_t)row_ptr[i], vb * (size_t)len);
            rp2[r + 1] = rp2[r] + len;
        }
        EncodeParams q = p;
        q.sigma = 0;
        std::string err = encode_csr(m, n, nnz, rp2.data(), c2.data(), v2.data(), dtype, q, c, dev);
        if (!err.empty()) return err;
        c.sigma = p.sigma;
        c.perm = std::move(perm);
        return "";
    }
    const int threads = thread_count(p.threads);
    // checks in row chunks; the error reported is the one a serial scan finds
    // first (the lowest failing row)
    {
        const int T = (int)std::max<int64_t>(1, std::min<int64_t>(threads, m / 65536 + 1));
        std::vector<int64_t> bad(T, -1);
        parallel_chunks(m, T, [&](int64_t b, int64_t e, int t) {
            for (int64_t i = b; i < e; ++i)
                if (row_ptr[i + 1] < row_ptr[i]) {
                    bad[t] = i;
                    return;
                }
        });
        for (int64_t i : bad)
            if (i >= 0) return fail("EINVAL", "row_ptr decreases at row " + std::to_string(i));
        std::vector<int64_t> brow(T, -1);
        std::vector<int> bkind(T, 0);
        // device inputs: the columns are checked on the device (keys)
        if (!(dev && dev->inputs_on_device())) parallel_chunks(m, T, [&](int64_t b, int64_t e, int t) {
            for (int64_t i = b; i < e; ++i)
                for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
                    const int kind = (col[q] < 0 || col[q] >= n) ? 1
                                     : (q > row_ptr[i] && col[q] < col[q - 1]) ? 2 : 0;
                    if (kind) {
                        brow[t] = i;
                        bkind[t] = kind;
                        return;
                    }
                }
        });
        for (int t = 0; t < T; ++t) {
            if (brow[t] < 0) continue;
            if (bkind[t] == 1)
                return fail("ERANGE", "column index out of range in row " + std::to_string(brow[t]));
            return fail("EUNSORTED", "columns not ascending in row " + std::to_string(brow[t]));
        }
    }
    c = Container();
    c.dtype = dtype;
    c.layout = p.layout;
    c.lane_nnz = p.layout == kLayoutNnz ? p.lane_nnz : 0;
    c.m = m;
    c.n = n;
    c.nnz = nnz;
    c.seed = p.seed;
    c.first_mode = p.first_mode;
    c.esc_mode = p.esc_mode;
    c.row_ptr.assign(row_ptr, row_ptr + m + 1);
    c.num_lanes = p.layout == kLayoutRow ? m : (nnz + p.lane_nnz - 1) / p.lane_nnz;
    c.num_waves = (c.num_lanes + kWave - 1) / kWave;

    // symbols: delta keys (with resets at row and lane starts) and value bits
    std::vector<uint64_t> dkey, vkey;
    std::vector<KeyCount> dhist, vhist;
    if (dev) {
        std::string err = dev->keys(c, col, vals, dhist, vhist);
        if (!err.empty()) return err;
    } else {
        dkey.resize(nnz);
        vkey.resize(nnz);
        std::vector<uint8_t> rowstart(nnz, 0);
        for (int64_t i = 0; i < m; ++i)
            if (row_ptr[i] < row_ptr[i + 1]) rowstart[row_ptr[i]] = 1;
        parallel_chunks(c.num_lanes, threads, [&](int64_t b, int64_t e, int) {
            for (int64_t l = b; l < e; ++l) {
                int64_t g0, cnt;
                c.lane_range(l, g0, cnt);
                for (int64_t t = 0; t < cnt; ++t) {
                    int64_t g = g0 + t;
                    if (t == 0 || rowstart[g]) {
                        const int64_t row = c.layout == kLayoutRow ? l : row_of(c.row_ptr, g);
                        dkey[g] = (uint32_t)col[g] - first_base(c.first_mode, (uint32_t)row);
                    } else {
                        dkey[g] = (uint64_t)(col[g] - col[g - 1]);
                    }
                }
            }
        });
        parallel_chunks(nnz, threads, [&](int64_t b, int64_t e, int) {
            if (dtype == kF64) {
                const uint64_t *v = (const uint64_t *)vals;
                for (int64_t g = b; g < e; ++g) vkey[g] = v[g];
            } else {
                const uint32_t *v = (const uint32_t *)vals;
                for (int64_t g = b; g < e; ++g) vkey[g] = v[g];
            }
        });
        dhist = histogram(dkey, threads);
        vhist = histogram(vkey, threads);
    }
    Fit dfit = fit_alphabet(dhist, 32, true, (int)p.max_mult, threads);
    Fit vfit = fit_alphabet(vhist, dtype == kF64 ? 64 : 32, false, (int)p.max_mult, threads);
    SlotMap dsm, vsm;
    build_table(dfit, p.seed, c.dtab, dsm);
    build_table(vfit, p.seed ^ 0xd1b54a32d192ed03ull, c.vtab, vsm);
    table_stats(dfit, nnz, c.dtab);
    table_stats(vfit, nnz, c.vtab);
    const int dpad = pad_symbol(c.dtab, dsm), vpad = pad_symbol(c.vtab, vsm);
    if (dev) {
        if (c.esc_mode != 0)
            return fail("EUNSUPPORTED", "the device encoder writes escapes to separate regions only");
        AlphabetMap da, va;
        auto fill = [](const SlotMap &sm, int pad, AlphabetMap &a) {
            a.hkey = sm.hkey;
            a.hval = sm.hval;
            a.esc = sm.esc_index;
            a.pad = pad;
            a.meta.resize(sm.mult.size());
            for (size_t s = 0; s < sm.mult.size(); ++s)
                a.meta[s] = (uint32_t)sm.first[s] | ((uint32_t)sm.mult[s] << 16);
            a.slots = sm.slots;
        };
        fill(dsm, dpad, da);
        fill(vsm, vpad, va);
        std::string err = dev->streams(da, va, c);
        if (!err.empty()) return err;
        if (c.word_off.size() != (size_t)c.num_waves + 1 || c.word_off.back() != c.words.size() ||
            c.escd_off.size() != (size_t)c.num_waves + 1 || c.escd_off.back() != c.escd.size() ||
            c.escv_off.size() != (size_t)c.num_waves + 1 || c.escv_off.back() != c.escv.size())
            return fail("ECORRUPT", "device encoder returned inconsistent offsets");
        return "";
    }

    // symbol indices per nonzero
    std::vector<int32_t> dsym(nnz), vsym(nnz);
    parallel_chunks(nnz, threads, [&](int64_t b, int64_t e, int) {
        for (int64_t g = b; g < e; ++g) {
            dsym[g] = dsm.lookup(dkey[g]);
            vsym[g] = vsm.lookup(vkey[g]);
        }
    });

    // waves in parallel chunks
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(threads, c.num_waves));
    std::vector<WaveOut> outs(T);
    parallel_chunks(c.num_waves, T, [&](int64_t wb, int64_t we, int tid) {
        WaveOut &o = outs[tid];
        std::vector<LaneCode> lanes(kWave);
        std::vector<int32_t> sym;
        int64_t g0s[kWave], cnts[kWave];
        for (int64_t w = wb; w < we; ++w) {
            o.woff.push_back(o.words.size());
            o.doff.push_back(o.escd.size());
            o.voff.push_back(o.escv.size());
            int64_t maxS = 0;
            for (int q = 0; q < kWave; ++q) {
                int64_t l = w * kWave + q;
                g0s[q] = 0;
                cnts[q] = 0;
                if (l < c.num_lanes) c.lane_range(l, g0s[q], cnts[q]);
                int64_t S = (cnts[q] + 3) / 4;
                sym.resize(8 * S);
                for (int64_t t = 0; t < 4 * S; ++t) {
                    if (t < cnts[q]) {
                        sym[2 * t] = dsym[g0s[q] + t];
                        sym[2 * t + 1] = vsym[g0s[q] + t];
                    } else {
                        sym[2 * t] = dpad;
                        sym[2 * t + 1] = vpad;
                    }
                }
                lanes[q] = LaneCode();
                encode_lane(sym.data(), S, dsm, vsm, lanes[q]);
                maxS = std::max(maxS, S);
            }
            for (int k = 0; k < 3; ++k)
                for (int q = 0; q < kWave; ++q)
                    if (lanes[q].S > 0) o.words.push_back(lanes[q].init[k]);
            const bool in_stream = c.esc_mode == 1;
            for (int64_t j = 0; j < maxS; ++j) {
                if (in_stream) {  // step j's escapes, read right after its table lookups
                    for (int k = 0; k < 4; ++k)
                        for (int q = 0; q < kWave; ++q) {
                            int64_t t = 4 * j + k;
                            if (t < cnts[q] && dsym[g0s[q] + t] == dsm.esc_index)
                                o.words.push_back((uint32_t)dkey[g0s[q] + t]);
                        }
                    for (int k = 0; k < 4; ++k)
                        for (int q = 0; q < kWave; ++q) {
                            int64_t t = 4 * j + k;
                            if (t < cnts[q] && vsym[g0s[q] + t] == vsm.esc_index) {
                                o.words.push_back((uint32_t)vkey[g0s[q] + t]);
                                if (c.dtype == kF64) o.words.push_back((uint32_t)(vkey[g0s[q] + t] >> 32));
                            }
                        }
                }
                if (j + 1 >= maxS) break;
                for (int q = 0; q < kWave; ++q)
                    if (j < lanes[q].S - 1 && lanes[q].load[2 * j]) o.words.push_back(lanes[q].w[3 * j]);
                for (int q = 0; q < kWave; ++q)
                    if (j < lanes[q].S - 1 && lanes[q].load[2 * j + 1])
                        o.words.push_back(lanes[q].w[3 * j + 1]);
                for (int q = 0; q < kWave; ++q)
                    if (j < lanes[q].S - 1) o.words.push_back(lanes[q].w[3 * j + 2]);
            }
            for (int64_t j = 0; j < maxS && !in_stream; ++j)
                for (int k = 0; k < 4; ++k)
                    for (int q = 0; q < kWave; ++q) {
                        int64_t t = 4 * j + k;
                        if (t < cnts[q] && dsym[g0s[q] + t] == dsm.esc_index)
                            o.escd.push_back((uint32_t)dkey[g0s[q] + t]);
                    }
            for (int64_t j = 0; j < maxS && !in_stream; ++j)
                for (int k = 0; k < 4; ++k)
                    for (int q = 0; q < kWave; ++q) {
                        int64_t t = 4 * j + k;
                        if (t < cnts[q] && vsym[g0s[q] + t] == vsm.esc_index)
                            o.escv.push_back(vkey[g0s[q] + t]);
                    }
        }
    });
    // concatenate
    c.word_off.reserve(c.num_waves + 1);
    for (auto &o : outs) {
        uint64_t wb = c.words.size(), db = c.escd.size(), vb = c.escv.size();
        for (size_t i = 0; i < o.woff.size(); ++i) {
            c.word_off.push_back(wb + o.woff[i]);
            c.escd_off.push_back(db + o.doff[i]);
            c.escv_off.push_back(vb + o.voff[i]);
        }
        c.words.insert(c.words.end(), o.words.begin(), o.words.end());
        c.escd.insert(c.escd.end(), o.escd.begin(), o.escd.end());
        c.escv.insert(c.escv.end(), o.escv.begin(), o.escv.end());
    }
    c.word_off.push_back(c.words.size());
    c.escd_off.push_back(c.escd.size());
    c.escv_off.push_back(c.escv.size());
    return "";
}

// ------------------------------------------------------------------ file I/O
namespace {
const size_t kHeader = 256;
size_t al8(size_t x) { return (x + 7) & ~(size_t)7; }

void put_table(std::vector<uint8_t> &b, size_t off, const Table &t) {
    for (int i = 0; i < kSlots; ++i) {
        uint8_t *e = &b[off + 16 * (size_t)i];
        if (!(t.flags[i] & 1)) continue;
        memcpy(e, &t.sym[i], 8);
        e[8] = t.digit[i];
        e[9] = (uint8_t)(t.base[i] - 1);
        e[10] = t.flags[i] & 3;
    }
}

// sym_bits: width of a table symbol (delta keys below 2^30 are checked
// separately; FP32 values are 32-bit patterns)
std::string get_table(const uint8_t *b, Table &t, bool is_delta, int sym_bits = 64) {
    t = Table();
    int counts[kSlots + 1];
    (void)counts;
    for (int i = 0; i < kSlots; ++i) {
        const uint8_t *e = b + 16 * (size_t)i;
        if (e[10] & ~3u) return fail("ECORRUPT", "bad slot flags");
        if (!(e[10] & 1)) continue;
        memcpy(&t.sym[i], e, 8);
        t.digit[i] = e[8];
        t.base[i] = (uint16_t)(e[9] + 1);
        t.flags[i] = e[10];
        if (t.digit[i] >= t.base[i]) return fail("ECORRUPT", "slot digit >= base");
        if (t.flags[i] & 2) {
            if (t.sym[i] != 0) return fail("ECORRUPT", "escape slot with a symbol");
            t.has_escape = true;
        } else if (is_delta && t.sym[i] >= kDeltaLimit) {
            return fail("ECORRUPT", "table delta above 2^30");
        } else if (sym_bits < 64 && (t.sym[i] >> sym_bits) != 0) {
            return fail("ECORRUPT", "table value wider than the value type");
        }
    }
    // every symbol must own exactly `base` slots with digits 0..base-1
    std::unordered_map<uint64_t, std::vector<int>> by;
    for (int i = 0; i < kSlots; ++i)
        if (t.flags[i] & 1) by[(t.flags[i] & 2) ? ~0ull : t.sym[i]].push_back(i);
    for (auto &kv : by) {
        int b0 = t.base[kv.second[0]];
        if ((int)kv.second.size() != b0) return fail("ECORRUPT", "symbol slot count != base");
        std::vector<uint8_t> seen(b0, 0);
        for (int i : kv.second) {
            if (t.base[i] != b0 || seen[t.digit[i]]) return fail("ECORRUPT", "inconsistent symbol slots");
            seen[t.digit[i]] = 1;
        }
        if (kv.first != ~0ull) t.symbols++;
    }
    return "";
}
}  // namespace

std::string save_container(const Container &c, const std::string &path) {
    const size_t vb = c.value_bytes();
    size_t sz = kHeader;
    const size_t o_dt = sz; sz = al8(sz + 16 * kSlots);
    const size_t o_vt = sz; sz = al8(sz + 16 * kSlots);
    const size_t o_rp = sz; sz = al8(sz + 4 * (size_t)(c.m + 1));
    const size_t o_wo = sz; sz = al8(sz + 8 * (size_t)(c.num_waves + 1));
    const size_t o_do = sz; sz = al8(sz + 8 * (size_t)(c.num_waves + 1));
    const size_t o_vo = sz; sz = al8(sz + 8 * (size_t)(c.num_waves + 1));
    const size_t o_w = sz; sz = al8(sz + 4 * c.words.size());
    const size_t o_ed = sz; sz = al8(sz + 4 * c.escd.size());
    const size_t o_ev = sz; sz = al8(sz + vb * c.escv.size());
    const size_t o_pm = sz; sz = al8(sz + (c.sigma ? 4 * (size_t)c.m : 0));
    std::vector<uint8_t> b(sz, 0);
    put_table(b, o_dt, c.dtab);
    put_table(b, o_vt, c.vtab);
    memcpy(&b[o_rp], c.row_ptr.data(), 4 * c.row_ptr.size());
    memcpy(&b[o_wo], c.word_off.data(), 8 * c.word_off.size());
    memcpy(&b[o_do], c.escd_off.data(), 8 * c.escd_off.size());
    memcpy(&b[o_vo], c.escv_off.data(), 8 * c.escv_off.size());
    if (!c.words.empty()) memcpy(&b[o_w], c.words.data(), 4 * c.words.size());
    if (!c.escd.empty()) memcpy(&b[o_ed], c.escd.data(), 4 * c.escd.size());
    for (size_t i = 0; i < c.escv.size(); ++i) {
        if (vb == 8) memcpy(&b[o_ev + 8 * i], &c.escv[i], 8);
        else { uint32_t x = (uint32_t)c.escv[i]; memcpy(&b[o_ev + 4 * i], &x, 4); }
    }
    if (c.sigma && c.m) memcpy(&b[o_pm], c.perm.data(), 4 * (size_t)c.m);
    memcpy(&b[0], "CSRDTANS", 8);
    uint32_t h32[4] = {1, c.dtype, c.layout, c.lane_nnz};
    memcpy(&b[8], h32, 16);
    int64_t h64[8] = {c.m, c.n, c.nnz, c.num_lanes, c.num_waves, (int64_t)c.words.size(),
                      (int64_t)c.escd.size(), (int64_t)c.escv.size()};
    memcpy(&b[24], h64, 64);
    memcpy(&b[88], &c.seed, 8);
    memcpy(&b[104], &c.first_mode, 4);
    memcpy(&b[108], &c.esc_mode, 4);
    memcpy(&b[112], &c.sigma, 4);
    uint64_t chk = fnv1a(b.data() + kHeader, sz - kHeader);
    memcpy(&b[96], &chk, 8);
    FILE *f = fopen(path.c_str(), "wb");
    if (!f) return fail("EIO", "cannot open " + path);
    size_t wr = fwrite(b.data(), 1, b.size(), f);
    int cl = fclose(f);
    if (wr != b.size() || cl != 0) return fail("EIO", "short write to " + path);
    return "";
}

std::string load_container(const std::string &path, Container &c) {
    FILE *f = fopen(path.c_str(), "rb");
    if (!f) return fail("EIO", "cannot open " + path);
    std::vector<uint8_t> b;
    fseek(f, 0, SEEK_END);
    long len = ftell(f);
    fseek(f, 0, SEEK_SET);
    if (len < (long)kHeader) { fclose(f); return fail("ECORRUPT", "file shorter than the header"); }
    b.resize((size_t)len);
    size_t rd = fread(b.data(), 1, b.size(), f);
    fclose(f);
    if (rd != b.size()) return fail("EIO", "short read from " + path);
    if (memcmp(b.data(), "CSRDTANS", 8) != 0) return fail("ECORRUPT", "bad magic");
    uint32_t h32[4];
    memcpy(h32, &b[8], 16);
    if (h32[0] != 1) return fail("ECORRUPT", "unsupported container version");
    int64_t h64[8];
    memcpy(h64, &b[24], 64);
    uint64_t chk;
    memcpy(&chk, &b[96], 8);
    if (fnv1a(b.data() + kHeader, b.size() - kHeader) != chk) return fail("ECORRUPT", "checksum mismatch");
    c = Container();
    c.dtype = h32[1];
    c.layout = h32[2];
    c.lane_nnz = h32[3];
    c.m = h64[0]; c.n = h64[1]; c.nnz = h64[2]; c.num_lanes = h64[3]; c.num_waves = h64[4];
    const int64_t nw = h64[5], nd = h64[6], nv = h64[7];
    memcpy(&c.seed, &b[88], 8);
    memcpy(&c.first_mode, &b[104], 4);
    memcpy(&c.esc_mode, &b[108], 4);
    memcpy(&c.sigma, &b[112], 4);
    if (c.dtype != kF32 && c.dtype != kF64) return fail("ECORRUPT", "bad dtype");
    if (c.first_mode > 1) return fail("ECORRUPT", "bad first-delta mode");
    if (c.esc_mode > 1 || (c.esc_mode == 1 && (nd != 0 || nv != 0))) return fail("ECORRUPT", "bad escape mode");
    if (c.sigma % kWave || (c.sigma && c.layout != kLayoutRow)) return fail("ECORRUPT", "bad row-sort window");
    if (c.layout != kLayoutRow && c.layout != kLayoutNnz) return fail("ECORRUPT", "bad layout");
    if (c.m < 0 || c.n < 0 || c.nnz < 0 || nw < 0 || nd < 0 || nv < 0 || c.m >= (1ll << 31) ||
        c.n >= (1ll << 31) || c.nnz >= (1ll << 31))
        return fail("ECORRUPT", "bad sizes");
    if (c.layout == kLayoutNnz && (c.lane_nnz == 0 || c.lane_nnz % 4)) return fail("ECORRUPT", "bad lane_nnz");
    int64_t lanes = c.layout == kLayoutRow ? c.m : (c.nnz + c.lane_nnz - 1) / c.lane_nnz;
    if (lanes != c.num_lanes || c.num_waves != (lanes + kWave - 1) / kWave) return fail("ECORRUPT", "bad lane counts");
    const size_t vb = c.value_bytes();
    size_t sz = kHeader;
    const size_t o_dt = sz; sz = al8(sz + 16 * kSlots);
    const size_t o_vt = sz; sz = al8(sz + 16 * kSlots);
    const size_t o_rp = sz; sz = al8(sz + 4 * (size_t)(c.m + 1));
    const size_t o_wo = sz; sz = al8(sz + 8 * (size_t)(c.num_waves + 1));
    const size_t o_do = sz; sz = al8(sz + 8 * (size_t)(c.num_waves + 1));
    const size_t o_vo = sz; sz = al8(sz + 8 * (size_t)(c.num_waves + 1));
    const size_t o_w = sz; sz = al8(sz + 4 * (size_t)nw);
    const size_t o_ed = sz; sz = al8(sz + 4 * (size_t)nd);
    const size_t o_ev = sz; sz = al8(sz + vb * (size_t)nv);
    const size_t o_pm = sz; sz = al8(sz + (c.sigma ? 4 * (size_t)c.m : 0));
    if (sz != b.size()) return fail("ECORRUPT", "file size does not match the header");
    std::string e = get_table(&b[o_dt], c.dtab, true);
    if (e.empty()) e = get_table(&b[o_vt], c.vtab, false, c.dtype == kF32 ? 32 : 64);
    if (!e.empty()) return e;
    c.row_ptr.resize(c.m + 1);
    memcpy(c.row_ptr.data(), &b[o_rp], 4 * (size_t)(c.m + 1));
    if (c.row_ptr[0] != 0 || c.row_ptr[c.m] != c.nnz) return fail("ECORRUPT", "bad row_ptr ends");
    for (int64_t i = 0; i < c.m; ++i)
        if (c.row_ptr[i + 1] < c.row_ptr[i]) return fail("ECORRUPT", "row_ptr decreases");
    c.word_off.resize(c.num_waves + 1);
    c.escd_off.resize(c.num_waves + 1);
    c.escv_off.resize(c.num_waves + 1);
    memcpy(c.word_off.data(), &b[o_wo], 8 * c.word_off.size());
    memcpy(c.escd_off.data(), &b[o_do], 8 * c.escd_off.size());
    memcpy(c.escv_off.data(), &b[o_vo], 8 * c.escv_off.size());
    auto mono = [](const std::vector<uint64_t> &v, int64_t total) {
        if (v.front() != 0 || v.back() != (uint64_t)total) return false;
        for (size_t i = 1; i < v.size(); ++i)
            if (v[i] < v[i - 1]) return false;
        return true;
    };
    if (!mono(c.word_off, nw) || !mono(c.escd_off, nd) || !mono(c.escv_off, nv))
        return fail("ECORRUPT", "bad per-wave offsets");
    c.words.resize(nw);
    c.escd.resize(nd);
    c.escv.resize(nv);
    if (nw) memcpy(c.words.data(), &b[o_w], 4 * (size_t)nw);
    if (nd) memcpy(c.escd.data(), &b[o_ed], 4 * (size_t)nd);
    for (int64_t i = 0; i < nv; ++i) {
        if (vb == 8) memcpy(&c.escv[i], &b[o_ev + 8 * i], 8);
        else { uint32_t x; memcpy(&x, &b[o_ev + 4 * i], 4); c.escv[i] = x; }
    }
    if (c.sigma) {
        // the stored order must be the sorted order of the original rows
        c.perm.resize(c.m);
        if (c.m) memcpy(c.perm.data(), &b[o_pm], 4 * (size_t)c.m);
        std::vector<int32_t> orp, chk;
        if (!original_row_ptr(c, orp)) return fail("ECORRUPT", "row order is not a permutation");
        sigma_order(c.m, orp.data(), c.sigma, chk);
        if (chk != c.perm) return fail("ECORRUPT", "rows are not in sorted order");
    }
    return "";
}

// ------------------------------------------------------- verifying decoder
// Decodes every wave with the same integer steps as the GPU kernels
// (dtans_core.hpp) and checks that each wave consumes exactly its words and
// escapes and that every slot used is a used table slot.
std::string host_decode(const Container &c, int32_t *colout, uint64_t *valout) {
    std::vector<uint8_t> rowstart(c.nnz, 0);
    for (int64_t i = 0; i < c.m; ++i)
        if (c.row_ptr[i] < c.row_ptr[i + 1]) rowstart[c.row_ptr[i]] = 1;
    std::vector<uint64_t> dm(kSlots);
    std::vector<uint8_t> used_d(kSlots), used_v(kSlots);
    for (int i = 0; i < kSlots; ++i) {
        uint64_t e = 0;
        if (c.dtab.flags[i] & 1) {
            e |= (c.dtab.flags[i] & 2) ? (1ull << 31) : (c.dtab.sym[i] & (kDeltaLimit - 1));
            e |= (uint64_t)((c.dtab.base[i] - 1) | (c.dtab.digit[i] << 8)) << 32;
        }
        if (c.vtab.flags[i] & 1) {
            if (c.vtab.flags[i] & 2) e |= 1ull << 30;
            e |= (uint64_t)((c.vtab.base[i] - 1) | (c.vtab.digit[i] << 8)) << 48;
        }
        dm[i] = e;
        used_d[i] = c.dtab.flags[i] & 1;
        used_v[i] = c.vtab.flags[i] & 1;
    }
    std::atomic<bool> bad(false);
    std::string first_error;
    const int T = thread_count(0);
    std::vector<std::string> errs(T);
    parallel_chunks(c.num_waves, T, [&](int64_t wb, int64_t we, int tid) {
        for (int64_t w = wb; w < we && !bad; ++w) {
            uint64_t wp = c.word_off[w], wend = c.word_off[w + 1];
            uint64_t dp = c.escd_off[w], dend = c.escd_off[w + 1];
            uint64_t vp = c.escv_off[w], vend = c.escv_off[w + 1];
            int64_t g0[kWave], cnt[kWave], S[kWave], maxS = 0;
            uint32_t w1[kWave], w2[kWave], w3[kWave], d[kWave], r[kWave], colv[kWave];
            for (int q = 0; q < kWave; ++q) {
                int64_t l = w * kWave + q;
                g0[q] = cnt[q] = 0;
                if (l < c.num_lanes) c.lane_range(l, g0[q], cnt[q]);
                S[q] = (cnt[q] + 3) / 4;
                maxS = std::max(maxS, S[q]);
                d[q] = 0; r[q] = 1; colv[q] = 0;
            }
            auto err = [&](const char *msg) {
                errs[tid] = fail("ECORRUPT", std::string(msg) + " in wave " + std::to_string(w));
                bad = true;
            };
            uint32_t *dst[3] = {w1, w2, w3};
            for (int k = 0; k < 3 && !bad; ++k)
                for (int q = 0; q < kWave; ++q)
                    if (S[q] > 0) {
                        if (wp >= wend) { err("stream overrun"); break; }
                        dst[k][q] = c.words[wp++];
                    }
            for (int64_t j = 0; j < maxS && !bad; ++j) {
                uint32_t sl[kWave][8];
                for (int q = 0; q < kWave; ++q)
                    if (j < S[q]) {
                        unpack8(w1[q], w2[q], w3[q], sl[q]);
                        for (int k = 0; k < 8; ++k)
                            if (!((k & 1) ? used_v : used_d)[sl[q][k]]) err("unused slot");
                    }
                if (bad) break;
                for (int k = 0; k < 4 && !bad; ++k)
                    for (int q = 0; q < kWave; ++q) {
                        int64_t t = 4 * j + k;
                        if (j >= S[q] || t >= cnt[q]) continue;
                        uint64_t e = dm[sl[q][2 * k]];
                        uint32_t delta = (uint32_t)e & (kDeltaLimit - 1);
                        if ((uint32_t)e >> 31 && c.esc_mode == 1) {
                            if (wp >= wend) { err("stream overrun"); break; }
                            delta = c.words[wp++];
                        } else if ((uint32_t)e >> 31) {
                            if (dp >= dend) { err("escape overrun"); break; }
                            delta = c.escd[dp++];
                        }
                        int64_t g = g0[q] + t;
                        uint64_t cc;
                        if (t == 0 || rowstart[g]) {
                            const int64_t row = c.layout == kLayoutRow ? w * kWave + q : row_of(c.row_ptr, g);
                            cc = (uint32_t)(first_base(c.first_mode, (uint32_t)row) + (uint32_t)delta);
                        } else {
                            cc = (uint64_t)colv[q] + delta;
                        }
                        if (cc >= (uint64_t)c.n) { err("column out of range"); break; }
                        colv[q] = (uint32_t)cc;
                        if (colout) colout[g] = (int32_t)cc;
                    }
                for (int k = 0; k < 4 && !bad; ++k)
                    for (int q = 0; q < kWave; ++q) {
                        int64_t t = 4 * j + k;
                        if (j >= S[q] || t >= cnt[q]) continue;
                        int s = sl[q][2 * k + 1];
                        uint64_t bits = c.vtab.sym[s];
                        if ((dm[s] >> 30) & 1 && c.esc_mode == 1) {
                            const int nwv = c.dtype == kF64 ? 2 : 1;
                            if (wp + nwv > wend) { err("stream overrun"); break; }
                            bits = c.words[wp++];
                            if (nwv == 2) bits |= (uint64_t)c.words[wp++] << 32;
                        } else if ((dm[s] >> 30) & 1) {
                            if (vp >= vend) { err("escape overrun"); break; }
                            bits = c.escv[vp++];
                        }
                        if (valout) valout[g0[q] + t] = bits;
                    }
                for (int g = 0; g < 2 && !bad; ++g)
                    for (int q = 0; q < kWave; ++q) {
                        if (j >= S[q] - 1) continue;
                        uint32_t D, Rm1, word = 0;
                        group4((uint32_t)(dm[sl[q][4 * g]] >> 32) & 0xffff,
                               (uint32_t)(dm[sl[q][4 * g + 1]] >> 48),
                               (uint32_t)(dm[sl[q][4 * g + 2]] >> 32) & 0xffff,
                               (uint32_t)(dm[sl[q][4 * g + 3]] >> 48), D, Rm1);
                        if (!append_and_check(d[q], r[q], D, Rm1, word)) {
                            if (wp >= wend) { err("stream overrun"); break; }
                            word = c.words[wp++];
                        }
                        (g == 0 ? w1 : w2)[q] = word;
                    }
                for (int q = 0; q < kWave && !bad; ++q)
                    if (j < S[q] - 1) {
                        if (wp >= wend) { err("stream overrun"); break; }
                        w3[q] = c.words[wp++];
                    }
            }
            if (!bad && (wp != wend || dp != dend || vp != vend)) err("stored and consumed sizes differ");
        }
    });
    for (auto &e : errs)
        if (!e.empty()) return e;
    return "";
}

// ------------------------------------------------------ layout NNZ metadata
void nnz_layout_meta(const Container &c, std::vector<int32_t> &lane_row,
                     std::vector<int32_t> &split_row, std::vector<int32_t> &split_first,
                     std::vector<int32_t> &split_last) {
    lane_row.assign(c.num_lanes, 0);
    split_row.clear();
    split_first.clear();
    split_last.clear();
    if (c.layout != kLayoutNnz) return;
    const int64_t T = c.lane_nnz;
    int64_t r = 0;
    for (int64_t l = 0; l < c.num_lanes; ++l) {
        int64_t g0 = l * T;
        while (r < c.m && c.row_ptr[r + 1] <= g0) ++r;  // row holding nonzero g0
        lane_row[l] = l == 0 ? 0 : (int32_t)r;
    }
    for (int64_t i = 0; i < c.m; ++i) {
        int64_t b = c.row_ptr[i], e = c.row_ptr[i + 1];
        if (e - b < 1) continue;
        int64_t la = b / T, lb = (e - 1) / T;
        if (la != lb) {
            split_row.push_back((int32_t)i);
            split_first.push_back((int32_t)la);
            split_last.push_back((int32_t)lb);
        }
    }
}

bool gpu_table(const Container &c, std::vector<uint64_t> &entry, std::vector<uint8_t> &values) {
    // column-delta table: delta | ((b - 1) | d << 16 | escape << 31) << 32;
    // value table: value bits, then b | d << 16 | escape << 31 (12 bytes per
    // slot for FP64, 8 for FP32); unused slots: b = 1, d = 0
    entry.assign(kSlots, 0);
    const size_t vb = c.value_bytes(), stride = vb + 4;
    values.assign(kSlots * stride, 0);
    bool direct = true;
    for (int i = 0; i < kSlots; ++i) {
        if (((c.dtab.flags[i] & 1) && c.dtab.base[i] > 255) || ((c.vtab.flags[i] & 1) && c.vtab.base[i] > 255))
            direct = false;
        uint64_t e = 0;
        if (c.dtab.flags[i] & 1) {
            const bool esc = (c.dtab.flags[i] & 2) != 0;
            const uint32_t meta = (c.dtab.base[i] - 1) | (c.dtab.digit[i] << 16) | (esc ? kMetaEscape : 0u);
            e = (esc ? 0u : (uint32_t)c.dtab.sym[i]) | ((uint64_t)meta << 32);
        }
        entry[i] = e;
        uint32_t vmeta = 1;
        uint8_t *dst = &values[stride * i];
        if (c.vtab.flags[i] & 1) {
            const bool esc = (c.vtab.flags[i] & 2) != 0;
            vmeta = c.vtab.base[i] | (c.vtab.digit[i] << 16) | (esc ? kMetaEscape : 0u);
            if (!esc) {
                if (vb == 8) memcpy(dst, &c.vtab.sym[i], 8);
                else { uint32_t x = (uint32_t)c.vtab.sym[i]; memcpy(dst, &x, 4); }
            }
        }
        memcpy(dst + vb, &vmeta, 4);
    }
    return direct;
}

}  // namespace dtans
