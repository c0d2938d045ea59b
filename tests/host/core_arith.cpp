// Host check of the digit-group arithmetic the decode kernels use with the
// device tables (dtans_core.hpp): a (delta, value) pair of symbols as one
// packed (base product, digit pair) and two pairs joined into a group, against
// the symbol-by-symbol definition of appending mixed-radix digits
// (D = ((d0 b1 + d1) b2 + d2) b3 + d3, R = b0 b1 b2 b3).  Direct tables
// (every base at most 255) on the 16-bit formulation, tables with bases up
// to 256 on the general one; bases 1, 2, 255, 256 and random ones.
#include <cstdio>
#include <cstdint>
#include <random>

#include "dtans_core.hpp"

using namespace dtans;

static uint32_t dmeta(uint32_t b, uint32_t d) { return (b - 1) | (d << 16); }
static uint32_t vmeta(uint32_t b, uint32_t d) { return b | (d << 16); }

int main() {
    std::mt19937_64 rng(12345);
    const uint32_t edge[] = {1, 2, 3, 16, 127, 254, 255};
    long fails = 0, checks = 0;
    auto pick = [&](uint32_t maxb) -> uint32_t {
        uint64_t u = rng();
        if (u % 4 == 0) {
            uint32_t e = edge[(u >> 8) % 7];
            return e <= maxb ? e : maxb;
        }
        return 1 + (uint32_t)((u >> 16) % maxb);
    };
    for (int it = 0; it < 2000000; ++it) {
        const bool general = it & 1;
        const uint32_t maxb = general ? 256 : 255;
        uint32_t b[4], d[4];
        for (int k = 0; k < 4; ++k) {
            b[k] = pick(maxb);
            d[k] = (uint32_t)(rng() % b[k]);
        }
        if (general && (it & 2))
            for (int k = 0; k < 4; ++k) { b[k] = 256; d[k] = (uint32_t)(rng() % 256); }
        // definition, 64-bit
        uint64_t Dref = 0, Rref = 1;
        for (int k = 0; k < 4; ++k) { Dref = Dref * b[k] + d[k]; Rref *= b[k]; }
        uint32_t D, R;
        ++checks;
        if (!general) {
            group_pairs_ref(pair_rd_ref(dmeta(b[0], d[0]), vmeta(b[1], d[1])),
                            pair_rd_ref(dmeta(b[2], d[2]), vmeta(b[3], d[3])), D, R);
            if (D != Dref || R != Rref) {
                if (fails++ < 5) std::printf("direct mismatch: D %u vs %llu, R %u vs %llu\n", D,
                                             (unsigned long long)Dref, R, (unsigned long long)Rref);
            }
        } else {
            uint32_t Rm1;
            group_general(dmeta(b[0], d[0]), vmeta(b[1], d[1]), dmeta(b[2], d[2]), vmeta(b[3], d[3]), D, Rm1);
            if (D != Dref || (uint64_t)Rm1 + 1 != Rref) {
                if (fails++ < 5) std::printf("general mismatch: D %u vs %llu, R-1 %u vs %llu\n", D,
                                             (unsigned long long)Dref, Rm1, (unsigned long long)Rref - 1);
            }
        }
        // the state update: the 64-bit products split at 2^32 exactly as the
        // 128-bit definition does
        const uint32_t r0 = 1 + (uint32_t)(rng() % 0xffffffffu), d0 = (uint32_t)(rng() % r0);
        if (!general) {
            uint32_t dd = d0, rr = r0, w = 0;
            const bool ex = append_word(dd, rr, D, R, w);
            const unsigned __int128 dfull = (unsigned __int128)d0 * R + D, rfull = (unsigned __int128)r0 * R;
            const bool exref = (rfull >> 32) != 0;
            const uint32_t dexp = exref ? (uint32_t)(dfull >> 32) : (uint32_t)dfull;
            const uint32_t rexp = exref ? (uint32_t)(rfull >> 32) : (uint32_t)rfull;
            if (ex != exref || dd != dexp || rr != rexp || (ex && w != (uint32_t)dfull)) {
                if (fails++ < 5) std::printf("append mismatch\n");
            }
        }
    }
    std::printf("%ld checks, %ld failures\n", checks, fails);
    return fails != 0;
}
