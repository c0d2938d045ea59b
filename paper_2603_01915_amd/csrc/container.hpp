// Host-side CSR-dtANS container of the library: the encoded matrix as it is
// written to / read from a file and uploaded to the GPU.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <array>
#include <string>
#include <vector>

#include "dtans_core.hpp"

namespace dtans {

enum : uint32_t { kF32 = 1, kF64 = 2 };
enum : uint32_t { kLayoutRow = 1, kLayoutNnz = 2 };

// One alphabet's coding table over K slots (Sec. III-D, IV-C): the symbol,
// digit and base of every slot; flags bit 0 = slot used, bit 1 = escape.
struct Table {
    std::array<uint64_t, kSlots> sym{};
    std::array<uint8_t, kSlots> digit{};
    std::array<uint16_t, kSlots> base{};  // 1..256, 0 when unused
    std::array<uint8_t, kSlots> flags{};
    int symbols = 0;        // table symbols without the escape
    bool has_escape = false;
    double entropy = 0, cross_entropy = 0;  // Eq. 1 / Eq. 2 over the encoded symbols
};

struct Container {
    uint32_t dtype = kF64, layout = kLayoutRow, lane_nnz = 0;
    uint32_t first_mode = 0;  // first delta of a row: 0 its column, 1 relative to the row
    // escaped symbols (Sec. IV-F): 0 in separate regions per wave (escd, escv);
    // 1 in the word stream, a decoding step's escaped deltas and then values
    // ((position, lane) order; FP64 values as two words, low first) between
    // the words read before that step and the words its checks read
    uint32_t esc_mode = 0;
    // row order (layout ROW): 0 = CSR order; else the encoded rows are the
    // original ones sorted by descending length within windows of sigma rows
    // (a SELL-C-sigma base, C = 64) and perm[r] is the original row of
    // encoded row r; row_ptr is then the encoded matrix's
    uint32_t sigma = 0;
    std::vector<int32_t> perm;
    int64_t m = 0, n = 0, nnz = 0, num_lanes = 0, num_waves = 0;
    uint64_t seed = 1;
    Table dtab, vtab;
    std::vector<int32_t> row_ptr;                 // m + 1
    std::vector<uint64_t> word_off, escd_off, escv_off;  // num_waves + 1 each
    std::vector<uint32_t> words;
    std::vector<uint32_t> escd;
    std::vector<uint64_t> escv;                   // FP32 values in the low 32 bits

    size_t value_bytes() const { return dtype == kF64 ? 8 : 4; }
    // nonzero range of lane l
    void lane_range(int64_t l, int64_t &g0, int64_t &cnt) const {
        if (layout == kLayoutRow) {
            g0 = row_ptr[l];
            cnt = (int64_t)row_ptr[l + 1] - row_ptr[l];
        } else {
            g0 = l * (int64_t)lane_nnz;
            int64_t e = g0 + lane_nnz;
            cnt = (e < nnz ? e : nnz) - g0;
        }
    }
};

// the (nonempty) row holding nonzero g: the last i with row_ptr[i] <= g
// SELL-C-sigma row order (Kreutzer et al. 2014): within each window of sigma
// rows, rows by descending number of nonzeros, ties in their original order;
// perm[r] = original row placed at r.
inline void sigma_order(int64_t m, const int32_t *row_ptr, uint32_t sigma, std::vector<int32_t> &perm) {
    perm.resize(m);
    for (int64_t i = 0; i < m; ++i) perm[i] = (int32_t)i;
    if (!sigma) return;
    for (int64_t w = 0; w < m; w += sigma) {
        auto b = perm.begin() + w, e = perm.begin() + std::min<int64_t>(m, w + sigma);
        std::stable_sort(b, e, [&](int32_t x, int32_t y) {
            return row_ptr[x + 1] - row_ptr[x] > row_ptr[y + 1] - row_ptr[y];
        });
    }
}

// Row pointers of the original matrix of a row-sorted container; false when
// perm is not a permutation of the rows.
inline bool original_row_ptr(const Container &c, std::vector<int32_t> &orp) {
    orp.assign(c.m + 1, 0);
    std::vector<uint8_t> seen(c.m, 0);
    for (int64_t r = 0; r < c.m; ++r) {
        const int32_t i = c.perm[r];
        if (i < 0 || i >= c.m || seen[i]) return false;
        seen[i] = 1;
        orp[i + 1] = c.row_ptr[r + 1] - c.row_ptr[r];
    }
    for (int64_t i = 0; i < c.m; ++i) orp[i + 1] += orp[i];
    return true;
}

inline int64_t row_of(const std::vector<int32_t> &row_ptr, int64_t g) {
    int64_t lo = 0, hi = (int64_t)row_ptr.size() - 1;  // row_ptr[lo] <= g < row_ptr[hi]
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if (row_ptr[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

struct EncodeParams {
    uint32_t layout = kLayoutRow;
    uint32_t lane_nnz = 0;
    uint32_t max_mult = 255;  // multiplicity cap, at most M = 256
    uint32_t first_mode = 1;  // Container::first_mode
    uint32_t esc_mode = 0;    // Container::esc_mode
    uint32_t sigma = 0;       // Container::sigma (layout ROW, a multiple of 64)
    uint64_t seed = 1;
    int threads = 0;  // 0 = hardware concurrency
};

// Count of one symbol key (histograms are sorted by key).
struct KeyCount {
    uint64_t key;
    int64_t count;
};

// The alphabets as the per-nonzero passes need them: an open-addressing map
// key -> symbol index (hkey / hval, hval -1 = empty, multiplicative hash of
// SlotMap::lookup; keys not found are the escape symbol esc), meta[s] = first
// logical slot of s | base of s << 16, slots[first + digit] = physical slot
// of that digit, and the padding symbol.
struct AlphabetMap {
    std::vector<uint64_t> hkey;
    std::vector<int32_t> hval;
    int32_t esc = -1, pad = -1;
    std::vector<uint32_t> meta;
    std::vector<uint16_t> slots;
};

// The per-nonzero passes of the encoder on a device (encode_kernels.hip):
// keys forms the delta and value keys of every nonzero (Container geometry
// already set; row_ptr validated on the host) and returns both histograms;
// with inputs_on_device() the col / vals pointers are device pointers, and
// keys also checks the columns (range, ascending within rows), returning the
// error a serial scan of the rows would find first;
// streams then maps every nonzero to its symbols and writes the words and
// escape regions of every wave, with their offsets, into the container
// (Sec. IV-B, IV-E, IV-F), exactly as the host passes would.
class DeviceEncoder {
  public:
    virtual ~DeviceEncoder() {}
    virtual std::string keys(const Container &c, const int32_t *col, const void *vals,
                             std::vector<KeyCount> &dhist, std::vector<KeyCount> &vhist) = 0;
    virtual std::string streams(const AlphabetMap &d, const AlphabetMap &v, Container &c) = 0;
    virtual bool inputs_on_device() const = 0;
};
// A DeviceEncoder on the current GPU running on `stream` (a hipStream_t);
// device_inputs: col and vals handed to encode_csr are device pointers.
DeviceEncoder *new_device_encoder(void *stream, bool device_inputs = false);

// All functions return an empty string on success or an error message whose
// first word is the error class ("EINVAL: ...", "ERANGE: ...", ...).
// With `dev`, the per-nonzero passes run there (validation, the alphabet
// fit and the tables stay on the host).
std::string encode_csr(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                       const int32_t *col, const void *vals, uint32_t dtype,
                       const EncodeParams &p, Container &out, DeviceEncoder *dev = nullptr);
std::string save_container(const Container &c, const std::string &path);
std::string load_container(const std::string &path, Container &c);
// Full host decode with the kernels' integer arithmetic; fills col / vals
// (value bits, FP32 in the low half) when non-null.
std::string host_decode(const Container &c, int32_t *col, uint64_t *vals);

// Layout NNZ metadata derived from row_ptr: the row holding each lane's first
// nonzero (lane 0 starts at row 0 so that leading empty rows are its own), and
// the rows that span more than one lane with their first and last lane.
void nnz_layout_meta(const Container &c, std::vector<int32_t> &lane_row,
                     std::vector<int32_t> &split_row, std::vector<int32_t> &split_first,
                     std::vector<int32_t> &split_last);

// Device tables (see dtans_core.hpp): one 64-bit column-delta entry per slot
// and one value entry per slot (value bits + metadata, 12 bytes for FP64, 8
// for FP32); returns true for "direct" tables (every base at most 255)
bool gpu_table(const Container &c, std::vector<uint64_t> &entry, std::vector<uint8_t> &values);

}  // namespace dtans
