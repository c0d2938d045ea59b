// Round trips of the library's host encoder for a sanitizer build (CPU only):
// seeded random and adversarial CSR matrices are encoded in both layouts and
// dtypes, written, read back (checksum and structure checks) and decoded by
// the host decoder, which must return the original columns and value bits.
// Exit status 0 when every case round-trips; the sanitizers abort otherwise.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "container.hpp"

using namespace dtans;

static uint64_t g_state = 0x1234567;
static uint64_t rnd() {  // splitmix64 (Steele, Lea, Flood)
    uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

struct Csr {
    int64_t m, n;
    std::vector<int32_t> rp, ci;
    std::vector<double> v;
};

static Csr random_csr(int64_t m, int64_t n, int maxlen, int pool, int empty_every) {
    Csr a{m, n, {0}, {}, {}};
    std::vector<double> vals(pool);
    for (auto &x : vals) x = (double)(int64_t)(rnd() % 2001 - 1000) / 64.0;
    for (int64_t i = 0; i < m; ++i) {
        int len = (empty_every && i % empty_every == 0) ? 0 : (int)(rnd() % (maxlen + 1));
        int64_t c = (int64_t)(rnd() % (uint64_t)n);
        for (int k = 0; k < len && c < n; ++k) {
            a.ci.push_back((int32_t)c);
            a.v.push_back(vals[rnd() % pool]);
            c += (int64_t)(rnd() % 5);  // duplicates (gap 0) allowed
        }
        a.rp.push_back((int32_t)a.ci.size());
    }
    return a;
}

static int check(const Csr &a, uint32_t dtype, uint32_t layout, uint32_t T, uint32_t cap, uint32_t first,
                 const char *path) {
    EncodeParams p;
    p.layout = layout;
    p.lane_nnz = T;
    p.max_mult = cap;
    p.first_mode = first;
    p.seed = rnd();
    p.threads = 3;
    std::vector<float> v32(a.v.begin(), a.v.end());
    const void *vals = dtype == kF64 ? (const void *)a.v.data() : (const void *)v32.data();
    Container c;
    std::string e = encode_csr(a.m, a.n, (int64_t)a.ci.size(), a.rp.data(), a.ci.data(), vals, dtype, p, c);
    if (!e.empty()) { printf("encode failed: %s\n", e.c_str()); return 1; }
    e = save_container(c, path);
    if (!e.empty()) { printf("save failed: %s\n", e.c_str()); return 1; }
    Container d;
    e = load_container(path, d);
    if (!e.empty()) { printf("load failed: %s\n", e.c_str()); return 1; }
    std::vector<int32_t> col(a.ci.size() + 1);
    std::vector<uint64_t> bits(a.ci.size() + 1);
    e = host_decode(d, col.data(), bits.data());
    if (!e.empty()) { printf("decode failed: %s\n", e.c_str()); return 1; }
    for (size_t g = 0; g < a.ci.size(); ++g) {
        uint64_t want = 0;
        if (dtype == kF64) memcpy(&want, &a.v[g], 8);
        else { uint32_t w; memcpy(&w, &v32[g], 4); want = w; }
        if (col[g] != a.ci[g] || bits[g] != want) {
            printf("mismatch at nonzero %zu\n", g);
            return 1;
        }
    }
    return 0;
}

int main(int argc, char **argv) {
    const char *path = argc > 1 ? argv[1] : "roundtrip.dtans";
    int fails = 0, cases = 0;
    const Csr mats[] = {
        random_csr(300, 500, 20, 40, 0),      // regular
        random_csr(517, 4000, 70, 3000, 7),   // many values: escapes, empty rows
        random_csr(64, 64, 3, 2, 3),          // tiny, two values
        random_csr(1, 10, 9, 1, 0),           // one row
        random_csr(200, 100000, 30, 5, 11),   // wide: large first deltas
    };
    for (const Csr &a : mats)
        for (uint32_t dtype : {kF64, kF32})
            for (uint32_t layout : {kLayoutRow, kLayoutNnz})
                for (uint32_t cap : {255u, 256u})
                    for (uint32_t first : {0u, 1u}) {
                        const uint32_t T = layout == kLayoutNnz ? 4 * (1 + (uint32_t)(rnd() % 40)) : 0;
                        fails += check(a, dtype, layout, T, cap, first, path);
                        ++cases;
                    }
    printf("%d cases, %d failures\n", cases, fails);
    return fails != 0;
}
