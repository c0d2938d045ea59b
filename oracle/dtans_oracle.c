/*
 * Oracle for CSR-dtANS sparse matrix-vector multiplication.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle: only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant generator with the HIP path; the
 * two meet only in the container file format, which each side reads and
 * writes with its own code.
 *
 * What it computes (paper: Schaetzle, Pegolotti, Pueschel, "Fast Entropy
 * Decoding for Sparse MVM on GPUs", 2026):
 *
 *   - y = alpha*A*x + beta*y from the original CSR arrays in double precision,
 *     by the textbook definition of SpMV (Sec. III-A, Fig. 2), plus the
 *     transposed product and the multi-vector product written the same way;
 *   - a reference dtANS encoder and decoder of the CSR-dtANS container:
 *     delta-encoding of column indices per row (Sec. IV-A), interleaved
 *     delta/value symbols per nonzero and 64-lane wave interleaving of the
 *     word streams (Sec. IV-B), tables of K = 4096 slots with multiplicity cap
 *     M = 256 (Sec. IV-C), decoding with W = 2^32, l = 8, o = 3, f = 2 one
 *     symbol at a time with a 128-bit state (Sec. IV-D, Alg. 3), the two-pass
 *     encoder (Sec. IV-E), escapes of rare symbols (Sec. IV-F) either to a
 *     separate region per wave or inside the word stream itself, read right
 *     after the decoding step that met them, the end-of-row load skipping
 *     and tail padding, and slot permutation (Sec. IV-F).
 *
 * Readings taken where the paper is silent (all listed in the design notes):
 * check g follows digit group g (symbols 1-4, then 5-8), digits are appended
 * as least significant, unpack takes w1 as most significant and i1 as the
 * lowest 12 bits, delta precedes value within a nonzero, escapes live in a
 * separate region per wave (or, in the in-stream mode, a step's escaped
 * deltas and then its escaped values, each in (position, lane) order, sit in
 * the word stream between the words read before the step and the words its
 * checks read; an FP64 value takes two words, low half first), and the last
 * segment of a lane stream performs no checks or loads.
 *
 * The multiplicity fit here is deliberately simple (proportional with a cap),
 * not the library's: any valid table decodes the same way.
 */
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define OK_SLOTS 4096     /* K */
#define OK_MCAP 256       /* M */
#define OK_WAVE 64        /* lanes per wave */
#define OK_NNZ_PER_SEG 4  /* l = 8 symbols = 4 (delta, value) pairs */
#define OK_HEADER 256
#define OK_DELTA_LIMIT (1u << 30) /* table deltas must be below this */

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_EIO = 2, ORC_ECORRUPT = 3, ORC_ENOMEM = 4 };

/* ======================================================================
 * SpMV family, plain definitions in double precision (Sec. III-A)
 *
 * Rows are independent, so the two products split their rows over the
 * threads set by oracle_set_threads (1 unless the caller asks for more); a
 * row's sum runs in the same order whatever the thread count.
 * ====================================================================== */

void oracle_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }

void oracle_csr_spmv_f64(int64_t m, const int32_t *row_ptr, const int32_t *col,
                         const double *val, const double *x, double *y,
                         double alpha, double beta)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
            s += val[p] * x[col[p]];
        y[i] = (beta == 0.0) ? alpha * s : alpha * s + beta * y[i];
    }
}

/* (|A| |x|)_i: the scale against which the tolerance on y is measured */
void oracle_csr_absmv_f64(int64_t m, const int32_t *row_ptr, const int32_t *col,
                          const double *val, const double *x, double *y)
{
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            double a = val[p] < 0 ? -val[p] : val[p];
            double b = x[col[p]] < 0 ? -x[col[p]] : x[col[p]];
            s += a * b;
        }
        y[i] = s;
    }
}

/* y (length n) = alpha * A^T x + beta * y, x of length m */
void oracle_csr_spmtv_f64(int64_t m, int64_t n, const int32_t *row_ptr,
                          const int32_t *col, const double *val, const double *x,
                          double *y, double alpha, double beta)
{
    double *acc = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
            acc[col[p]] += val[p] * x[i];
    for (int64_t j = 0; j < n; ++j)
        y[j] = (beta == 0.0) ? alpha * acc[j] : alpha * acc[j] + beta * y[j];
    free(acc);
}

/* Y (m x k, row-major, leading dim ldy) = alpha*A*X + beta*Y, X (n x k, ldx) */
void oracle_csr_spmm_f64(int64_t m, int64_t k, const int32_t *row_ptr,
                         const int32_t *col, const double *val, const double *X,
                         int64_t ldx, double *Y, int64_t ldy, double alpha,
                         double beta)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t c = 0; c < k; ++c) {
            double s = 0.0;
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                s += val[p] * X[(int64_t)col[p] * ldx + c];
            double *yy = &Y[i * ldy + c];
            *yy = (beta == 0.0) ? alpha * s : alpha * s + beta * *yy;
        }
}

/* ======================================================================
 * small helpers: FNV-1a 64 checksum, splitmix64 generator
 * ====================================================================== */

static uint64_t fnv1a64(const uint8_t *p, size_t n)
{
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

static uint64_t splitmix64(uint64_t *s)
{
    uint64_t z = (*s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* ======================================================================
 * coding tables (Sec. III-D, IV-C)
 * ====================================================================== */

typedef struct {
    uint64_t sym[OK_SLOTS];
    uint8_t digit[OK_SLOTS];
    uint16_t base[OK_SLOTS];    /* 1..256; 0 for an unused slot */
    uint8_t esc[OK_SLOTS];      /* 1 for slots of the escape symbol */
    /* encoder side: symbols in table order and their slots by digit */
    int nsym;                   /* number of table symbols incl. the escape */
    int esc_index;              /* index of the escape symbol or -1 */
    uint64_t keys[OK_SLOTS];    /* key of table symbol s (escape: unused) */
    int mult[OK_SLOTS];
    int *slot_by_digit[OK_SLOTS];
} otable;

static void otable_free(otable *t)
{
    for (int s = 0; s < t->nsym; ++s) free(t->slot_by_digit[s]);
    t->nsym = 0;
}

typedef struct { uint64_t key; int64_t count; } kc;

static int cmp_key(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

static int cmp_count_desc(const void *a, const void *b)
{
    const kc *x = (const kc *)a, *y = (const kc *)b;
    if (x->count != y->count) return x->count > y->count ? -1 : 1;
    return x->key < y->key ? -1 : x->key > y->key;
}

/* Build one alphabet's table from a multiset of keys.  Top keys (by count)
 * up to a fixed number get table slots with multiplicities proportional to
 * their counts (at least 1, at most M); the rest share one escape symbol.
 * Slots are laid out symbol by symbol and then shuffled (Sec. IV-F). */
static int build_table(otable *t, const uint64_t *keys, int64_t nkeys,
                       int is_delta, uint64_t seed)
{
    memset(t, 0, sizeof(*t));
    t->esc_index = -1;
    if (nkeys == 0) return ORC_OK;
    uint64_t *sorted = (uint64_t *)malloc((size_t)nkeys * sizeof(uint64_t));
    if (!sorted) return ORC_ENOMEM;
    memcpy(sorted, keys, (size_t)nkeys * sizeof(uint64_t));
    qsort(sorted, (size_t)nkeys, sizeof(uint64_t), cmp_key);
    int64_t ndistinct = 0;
    for (int64_t i = 0; i < nkeys; ++i)
        if (i == 0 || sorted[i] != sorted[i - 1]) ++ndistinct;
    kc *h = (kc *)malloc((size_t)ndistinct * sizeof(kc));
    int64_t q = -1;
    for (int64_t i = 0; i < nkeys; ++i) {
        if (i == 0 || sorted[i] != sorted[i - 1]) { ++q; h[q].key = sorted[i]; h[q].count = 0; }
        h[q].count++;
    }
    free(sorted);
    qsort(h, (size_t)ndistinct, sizeof(kc), cmp_count_desc);

    const int max_table = 2048;
    int ntab = 0;
    int64_t esc_count = 0;
    for (int64_t i = 0; i < ndistinct; ++i) {
        int fits = ntab < max_table && (!is_delta || h[i].key < OK_DELTA_LIMIT);
        if (fits) {
            t->keys[ntab] = h[i].key;
            t->mult[ntab] = (int)(h[i].count > 0x7fffffff ? 0x7fffffff : h[i].count);
            ++ntab;
        } else {
            esc_count += h[i].count;
        }
    }
    free(h);
    if (ntab == 0) { /* keep one ordinary symbol so that padding has one */
        t->keys[0] = 0;
        t->mult[0] = 0;
        ntab = 1;
    }
    int nsym = ntab + (esc_count > 0 ? 1 : 0);
    int64_t total = esc_count;
    for (int s = 0; s < ntab; ++s) total += t->mult[s];
    int64_t counts[OK_SLOTS];
    for (int s = 0; s < ntab; ++s) counts[s] = t->mult[s];
    if (esc_count > 0) { counts[ntab] = esc_count; t->esc_index = ntab; }
    /* proportional multiplicities, clamped to [1, M] */
    int64_t sum = 0;
    for (int s = 0; s < nsym; ++s) {
        int64_t mm = total > 0 ? (counts[s] * OK_SLOTS) / total : 1;
        if (mm < 1) mm = 1;
        if (mm > OK_MCAP) mm = OK_MCAP;
        t->mult[s] = (int)mm;
        sum += mm;
    }
    while (sum > OK_SLOTS) { /* shrink the largest multiplicity */
        int big = 0;
        for (int s = 1; s < nsym; ++s) if (t->mult[s] > t->mult[big]) big = s;
        t->mult[big]--;
        sum--;
    }
    t->nsym = nsym;
    /* logical layout: symbol after symbol, digits 0..m-1 */
    int perm[OK_SLOTS];
    for (int i = 0; i < OK_SLOTS; ++i) perm[i] = i;
    uint64_t st = seed;
    for (int i = OK_SLOTS - 1; i > 0; --i) {
        int j = (int)(splitmix64(&st) % (uint64_t)(i + 1));
        int tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
    }
    int logical = 0;
    for (int s = 0; s < nsym; ++s) {
        t->slot_by_digit[s] = (int *)malloc((size_t)t->mult[s] * sizeof(int));
        for (int d = 0; d < t->mult[s]; ++d) {
            int slot = perm[logical++];
            t->slot_by_digit[s][d] = slot;
            t->sym[slot] = (s == t->esc_index) ? 0 : t->keys[s];
            t->digit[slot] = (uint8_t)d;
            t->base[slot] = (uint16_t)t->mult[s];
            t->esc[slot] = (s == t->esc_index);
        }
    }
    return ORC_OK;
}

/* table symbol index of a key: binary search over the table symbols */
static int symbol_index(const otable *t, const int *order, uint64_t key)
{
    int ntab = t->esc_index >= 0 ? t->nsym - 1 : t->nsym;
    int lo = 0, hi = ntab - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        uint64_t k = t->keys[order[mid]];
        if (k == key) return order[mid];
        if (k < key) lo = mid + 1; else hi = mid - 1;
    }
    return t->esc_index; /* escaped */
}

static const otable *g_sort_table; /* qsort context (the oracle is serial) */
static int cmp_order(const void *a, const void *b)
{
    uint64_t x = g_sort_table->keys[*(const int *)a], y = g_sort_table->keys[*(const int *)b];
    return x < y ? -1 : x > y;
}

/* ======================================================================
 * container layout
 * ====================================================================== */

typedef struct {
    uint32_t dtype;    /* 1 = FP32, 2 = FP64 */
    uint32_t layout;   /* 1 = one row per lane, 2 = T nonzeros per lane */
    uint32_t lane_nnz; /* T for layout 2 */
    int64_t m, n, nnz, num_lanes, num_waves, n_words, n_escd, n_escv;
    uint64_t seed;
    uint32_t first_mode; /* first delta of a row: 0 its column, 1 column - row + 2^29 */
    uint32_t esc_mode;   /* escaped symbols: 0 separate regions, 1 in the word stream */
    uint32_t sigma;      /* 0: rows in their order; else rows sorted within windows of sigma */
} ohdr;

/* First delta of a row (or of a lane starting inside a row), mode 1: the
 * column minus the row plus 2^29, modulo 2^32 (an extension of the format:
 * the paper's first delta is the column itself, Sec. IV-A). */
#define ORC_FIRST_BIAS (1u << 29)
static uint32_t first_base(uint32_t mode, int64_t row)
{
    return mode ? (uint32_t)row - ORC_FIRST_BIAS : 0u;
}

/* the row holding nonzero g: the last i with row_ptr[i] <= g */
static int64_t row_of(const int32_t *row_ptr, int64_t m, int64_t g)
{
    int64_t lo = 0, hi = m; /* row_ptr[lo] <= g < row_ptr[hi] */
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if (row_ptr[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

static size_t align8(size_t x) { return (x + 7) & ~(size_t)7; }

/* lane geometry: nonzero range of lane `l` */
static void lane_range(const ohdr *H, const int32_t *row_ptr, int64_t l,
                       int64_t *g0, int64_t *cnt)
{
    if (H->layout == 1) {
        *g0 = row_ptr[l];
        *cnt = (int64_t)row_ptr[l + 1] - row_ptr[l];
    } else {
        *g0 = l * (int64_t)H->lane_nnz;
        int64_t e = *g0 + H->lane_nnz;
        if (e > H->nnz) e = H->nnz;
        *cnt = e - *g0;
    }
}

/* row_start[g] = 1 when nonzero g is the first nonzero of its row */
static uint8_t *row_start_flags(int64_t m, int64_t nnz, const int32_t *row_ptr)
{
    uint8_t *f = (uint8_t *)calloc((size_t)(nnz > 0 ? nnz : 1), 1);
    for (int64_t i = 0; i < m; ++i)
        if (row_ptr[i] < row_ptr[i + 1]) f[row_ptr[i]] = 1;
    return f;
}

/* ======================================================================
 * encoder (Sec. IV-E): base pass forward, digit pass backward
 * ====================================================================== */

typedef struct {
    int64_t S;            /* segments */
    uint32_t init[3];     /* w1 w2 w3 read before segment 0 */
    uint8_t *load1, *load2; /* per step j < S-1: 1 = conditional load */
    uint32_t *w1, *w2, *w3; /* per step j < S-1: the words for segment j+1 */
} olane;

static void unpack8(const uint32_t w[3], int slot[8])
{
    u128 V = ((u128)w[0] << 64) | ((u128)w[1] << 32) | (u128)w[2];
    for (int t = 0; t < 8; ++t) {
        slot[t] = (int)(V & 0xfff);
        V >>= 12;
    }
}

static void pack8(const int slot[8], uint32_t w[3])
{
    u128 V = 0;
    for (int t = 7; t >= 0; --t) V = (V << 12) | (u128)(slot[t] & 0xfff);
    w[2] = (uint32_t)V;
    w[1] = (uint32_t)(V >> 32);
    w[0] = (uint32_t)(V >> 64);
}

/* sym[2*t] = delta symbol index, sym[2*t+1] = value symbol index of nonzero t,
 * already padded to 4*S nonzeros */
static int encode_lane(olane *L, const int *sym, int64_t S, const otable *td,
                       const otable *tv)
{
    memset(L, 0, sizeof(*L));
    L->S = S;
    if (S == 0) return ORC_OK;
    int64_t steps = S - 1;
    size_t ns = (size_t)(steps > 0 ? steps : 1);
    L->load1 = (uint8_t *)calloc(ns, 1);
    L->load2 = (uint8_t *)calloc(ns, 1);
    L->w1 = (uint32_t *)calloc(ns, 4);
    L->w2 = (uint32_t *)calloc(ns, 4);
    L->w3 = (uint32_t *)calloc(ns, 4);
    /* base pass: radix only */
    u128 r = 1;
    for (int64_t j = 0; j < steps; ++j) {
        for (int g = 0; g < 2; ++g) {
            for (int t = 4 * g; t < 4 * g + 4; ++t) {
                const otable *T = (t % 2 == 0) ? td : tv;
                r *= (u128)T->mult[sym[8 * j + t]];
            }
            int extract = r >= ((u128)1 << 32);
            if (extract) r >>= 32;
            if (g == 0) L->load1[j] = !extract; else L->load2[j] = !extract;
        }
    }
    /* digit pass, backwards; the state after the last checks is 0 and the
     * last segment's digits are free (taken as 0) */
    int slots[8];
    for (int t = 0; t < 8; ++t) {
        const otable *T = (t % 2 == 0) ? td : tv;
        slots[t] = T->slot_by_digit[sym[8 * (S - 1) + t]][0];
    }
    u128 d = 0;
    for (int64_t j = steps - 1; j >= 0; --j) {
        uint32_t nxt[3];
        pack8(slots, nxt);
        L->w1[j] = nxt[0];
        L->w2[j] = nxt[1];
        L->w3[j] = nxt[2];
        int prev[8];
        for (int g = 1; g >= 0; --g) {
            uint8_t load = g == 0 ? L->load1[j] : L->load2[j];
            if (!load) d = (d << 32) | (u128)nxt[g];
            for (int t = 4 * g + 3; t >= 4 * g; --t) {
                const otable *T = (t % 2 == 0) ? td : tv;
                int s = sym[8 * j + t];
                u128 b = (u128)T->mult[s];
                int dig = (int)(d % b);
                d /= b;
                prev[t] = T->slot_by_digit[s][dig];
            }
        }
        memcpy(slots, prev, sizeof(slots));
    }
    if (d != 0) return ORC_EINVAL; /* cannot happen for a valid table */
    pack8(slots, L->init);
    return ORC_OK;
}

static void olane_free(olane *L)
{
    free(L->load1); free(L->load2); free(L->w1); free(L->w2); free(L->w3);
    memset(L, 0, sizeof(*L));
}

/* dynamic u32/u64 arrays */
typedef struct { uint64_t *p; int64_t n, cap; } vec64;
static void v64_push(vec64 *v, uint64_t x)
{
    if (v->n == v->cap) {
        v->cap = v->cap ? 2 * v->cap : 1024;
        v->p = (uint64_t *)realloc(v->p, (size_t)v->cap * 8);
    }
    v->p[v->n++] = x;
}

static void put_u32(uint8_t *b, uint32_t x) { memcpy(b, &x, 4); }
static void put_u64(uint8_t *b, uint64_t x) { memcpy(b, &x, 8); }
static uint32_t get_u32(const uint8_t *b) { uint32_t x; memcpy(&x, b, 4); return x; }
static uint64_t get_u64(const uint8_t *b) { uint64_t x; memcpy(&x, b, 8); return x; }

static void write_table(uint8_t *b, const otable *t)
{
    for (int i = 0; i < OK_SLOTS; ++i) {
        uint8_t *e = b + 16 * (size_t)i;
        memset(e, 0, 16);
        if (t->base[i] == 0) continue;
        put_u64(e, t->sym[i]);
        e[8] = t->digit[i];
        e[9] = (uint8_t)(t->base[i] - 1);
        e[10] = (uint8_t)(1 | (t->esc[i] ? 2 : 0));
    }
}

/*
 * Encode a CSR matrix into a container file.  dtype 1: vals are float,
 * dtype 2: vals are double.  layout 1: one row per lane; layout 2: lane_nnz
 * (multiple of 4) nonzeros per lane.  Columns must be sorted within rows.
 */
static int encode_rows(const char *path, int64_t m, int64_t n, int64_t nnz,
                       const int32_t *row_ptr, const int32_t *col, const void *vals,
                       int dtype, int layout, int lane_nnz, uint64_t seed, int first_mode, int esc_mode,
                       uint32_t sigma, const int32_t *perm)
{
    if (m < 0 || n < 0 || nnz < 0 || (dtype != 1 && dtype != 2) ||
        (layout != 1 && layout != 2) || (first_mode != 0 && first_mode != 1) ||
        (esc_mode != 0 && esc_mode != 1) ||
        (layout == 2 && (lane_nnz <= 0 || lane_nnz % 4 != 0)))
        return ORC_EINVAL;
    if (row_ptr[0] != 0 || row_ptr[m] != nnz) return ORC_EINVAL;
    for (int64_t i = 0; i < m; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) return ORC_EINVAL;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            if (col[p] < 0 || col[p] >= n) return ORC_EINVAL;
            if (p > row_ptr[i] && col[p] < col[p - 1]) return ORC_EINVAL;
        }
    }
    ohdr H;
    memset(&H, 0, sizeof(H));
    H.dtype = (uint32_t)dtype;
    H.layout = (uint32_t)layout;
    H.lane_nnz = layout == 2 ? (uint32_t)lane_nnz : 0;
    H.m = m; H.n = n; H.nnz = nnz; H.seed = seed; H.first_mode = (uint32_t)first_mode;
    H.esc_mode = (uint32_t)esc_mode;
    H.sigma = sigma;
    H.num_lanes = layout == 1 ? m : (nnz + lane_nnz - 1) / lane_nnz;
    H.num_waves = (H.num_lanes + OK_WAVE - 1) / OK_WAVE;

    /* symbols: delta (column difference within row and lane) and value bits */
    uint8_t *first = row_start_flags(m, nnz, row_ptr);
    size_t nz = (size_t)(nnz > 0 ? nnz : 1);
    uint64_t *dkey = (uint64_t *)malloc(nz * 8), *vkey = (uint64_t *)malloc(nz * 8);
    for (int64_t l = 0; l < H.num_lanes; ++l) {
        int64_t g0, c;
        lane_range(&H, row_ptr, l, &g0, &c);
        for (int64_t t = 0; t < c; ++t) {
            int64_t g = g0 + t;
            if (t == 0 || first[g])
                dkey[g] = (uint32_t)col[g] - first_base(H.first_mode, row_of(row_ptr, m, g));
            else
                dkey[g] = (uint64_t)(col[g] - col[g - 1]);
        }
    }
    for (int64_t g = 0; g < nnz; ++g) {
        if (dtype == 2) { uint64_t b; memcpy(&b, (const double *)vals + g, 8); vkey[g] = b; }
        else { uint32_t b; memcpy(&b, (const float *)vals + g, 4); vkey[g] = b; }
    }
    static otable td, tv; /* large; not reentrant (the oracle is serial) */
    int rc = build_table(&td, dkey, nnz, 1, seed);
    if (rc == ORC_OK) rc = build_table(&tv, vkey, nnz, 0, seed ^ 0x5bd1e995u);
    if (rc != ORC_OK) { free(first); free(dkey); free(vkey); return rc; }
    int *dord = (int *)malloc(sizeof(int) * OK_SLOTS), *vord = (int *)malloc(sizeof(int) * OK_SLOTS);
    int dn = td.esc_index >= 0 ? td.nsym - 1 : td.nsym;
    int vn = tv.esc_index >= 0 ? tv.nsym - 1 : tv.nsym;
    for (int s = 0; s < dn; ++s) dord[s] = s;
    for (int s = 0; s < vn; ++s) vord[s] = s;
    g_sort_table = &td; qsort(dord, (size_t)dn, sizeof(int), cmp_order);
    g_sort_table = &tv; qsort(vord, (size_t)vn, sizeof(int), cmp_order);
    /* padding (the decoder ignores padded nonzeros): the symbol on the
     * lowest-numbered used slot that is not the escape */
    int dpad = -1, vpad = -1;
    for (int i = OK_SLOTS - 1; i >= 0; --i) {
        if (td.base[i] && !td.esc[i]) dpad = symbol_index(&td, dord, td.sym[i]);
        if (tv.base[i] && !tv.esc[i]) vpad = symbol_index(&tv, vord, tv.sym[i]);
    }

    vec64 words = {0}, escd = {0}, escv = {0};
    uint64_t *woff = (uint64_t *)calloc((size_t)H.num_waves + 1, 8);
    uint64_t *doff = (uint64_t *)calloc((size_t)H.num_waves + 1, 8);
    uint64_t *voff = (uint64_t *)calloc((size_t)H.num_waves + 1, 8);
    olane lanes[OK_WAVE];
    int64_t lane_g0[OK_WAVE], lane_c[OK_WAVE];
    int *sym = NULL;
    size_t symcap = 0;
    for (int64_t w = 0; w < H.num_waves && rc == ORC_OK; ++w) {
        woff[w] = (uint64_t)words.n; doff[w] = (uint64_t)escd.n; voff[w] = (uint64_t)escv.n;
        int64_t maxS = 0;
        for (int q = 0; q < OK_WAVE; ++q) {
            int64_t l = w * OK_WAVE + q;
            lane_g0[q] = 0; lane_c[q] = 0;
            if (l < H.num_lanes) lane_range(&H, row_ptr, l, &lane_g0[q], &lane_c[q]);
            int64_t S = (lane_c[q] + 3) / 4;
            if ((size_t)(8 * S) > symcap) {
                symcap = (size_t)(8 * S);
                sym = (int *)realloc(sym, symcap * sizeof(int));
            }
            for (int64_t t = 0; t < 4 * S; ++t) {
                if (t < lane_c[q]) {
                    int64_t g = lane_g0[q] + t;
                    sym[2 * t] = symbol_index(&td, dord, dkey[g]);
                    sym[2 * t + 1] = symbol_index(&tv, vord, vkey[g]);
                } else {
                    sym[2 * t] = dpad;
                    sym[2 * t + 1] = vpad;
                }
            }
            rc = encode_lane(&lanes[q], sym, S, &td, &tv);
            if (rc != ORC_OK) break;
            if (S > maxS) maxS = S;
        }
        if (rc != ORC_OK) break;
        /* interleave: three initial rounds, then per step check 1, check 2,
         * unconditional, each in lane order over the lanes still running;
         * in the in-stream mode each step's escapes come first */
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < OK_WAVE; ++q)
                if (lanes[q].S > 0) v64_push(&words, lanes[q].init[r]);
        for (int64_t j = 0; j < maxS; ++j) {
            if (esc_mode == 1) {
                for (int pos = 0; pos < 4; ++pos)
                    for (int q = 0; q < OK_WAVE; ++q) {
                        int64_t t = 4 * j + pos;
                        if (t >= lane_c[q]) continue;
                        int64_t g = lane_g0[q] + t;
                        if (symbol_index(&td, dord, dkey[g]) == td.esc_index) v64_push(&words, dkey[g]);
                    }
                for (int pos = 0; pos < 4; ++pos)
                    for (int q = 0; q < OK_WAVE; ++q) {
                        int64_t t = 4 * j + pos;
                        if (t >= lane_c[q]) continue;
                        int64_t g = lane_g0[q] + t;
                        if (symbol_index(&tv, vord, vkey[g]) != tv.esc_index) continue;
                        v64_push(&words, vkey[g] & 0xffffffffu);
                        if (dtype == 2) v64_push(&words, vkey[g] >> 32);
                    }
            }
            if (j + 1 >= maxS) break;
            for (int q = 0; q < OK_WAVE; ++q)
                if (j < lanes[q].S - 1 && lanes[q].load1[j]) v64_push(&words, lanes[q].w1[j]);
            for (int q = 0; q < OK_WAVE; ++q)
                if (j < lanes[q].S - 1 && lanes[q].load2[j]) v64_push(&words, lanes[q].w2[j]);
            for (int q = 0; q < OK_WAVE; ++q)
                if (j < lanes[q].S - 1) v64_push(&words, lanes[q].w3[j]);
        }
        /* escapes: per segment, per nonzero position, in lane order */
        for (int64_t j = 0; j < maxS && esc_mode == 0; ++j)
            for (int pos = 0; pos < 4; ++pos)
                for (int q = 0; q < OK_WAVE; ++q) {
                    int64_t t = 4 * j + pos;
                    if (t >= lane_c[q]) continue;
                    int64_t g = lane_g0[q] + t;
                    if (symbol_index(&td, dord, dkey[g]) == td.esc_index) v64_push(&escd, dkey[g]);
                }
        for (int64_t j = 0; j < maxS && esc_mode == 0; ++j)
            for (int pos = 0; pos < 4; ++pos)
                for (int q = 0; q < OK_WAVE; ++q) {
                    int64_t t = 4 * j + pos;
                    if (t >= lane_c[q]) continue;
                    int64_t g = lane_g0[q] + t;
                    if (symbol_index(&tv, vord, vkey[g]) == tv.esc_index) v64_push(&escv, vkey[g]);
                }
        for (int q = 0; q < OK_WAVE; ++q) olane_free(&lanes[q]);
    }
    free(sym);
    woff[H.num_waves] = (uint64_t)words.n;
    doff[H.num_waves] = (uint64_t)escd.n;
    voff[H.num_waves] = (uint64_t)escv.n;
    H.n_words = words.n; H.n_escd = escd.n; H.n_escv = escv.n;

    if (rc == ORC_OK) {
        size_t vsz = dtype == 2 ? 8 : 4;
        size_t sz = OK_HEADER;
        sz = align8(sz + 16 * OK_SLOTS);
        sz = align8(sz + 16 * OK_SLOTS);
        sz = align8(sz + 4 * (size_t)(m + 1));
        sz = align8(sz + 8 * (size_t)(H.num_waves + 1));
        sz = align8(sz + 8 * (size_t)(H.num_waves + 1));
        sz = align8(sz + 8 * (size_t)(H.num_waves + 1));
        sz = align8(sz + 4 * (size_t)H.n_words);
        sz = align8(sz + 4 * (size_t)H.n_escd);
        sz = align8(sz + vsz * (size_t)H.n_escv);
        if (sigma) sz = align8(sz + 4 * (size_t)m);
        uint8_t *buf = (uint8_t *)calloc(sz, 1);
        size_t o = OK_HEADER;
        write_table(buf + o, &td); o = align8(o + 16 * OK_SLOTS);
        write_table(buf + o, &tv); o = align8(o + 16 * OK_SLOTS);
        memcpy(buf + o, row_ptr, 4 * (size_t)(m + 1)); o = align8(o + 4 * (size_t)(m + 1));
        for (int64_t w = 0; w <= H.num_waves; ++w) put_u64(buf + o + 8 * w, woff[w]);
        o = align8(o + 8 * (size_t)(H.num_waves + 1));
        for (int64_t w = 0; w <= H.num_waves; ++w) put_u64(buf + o + 8 * w, doff[w]);
        o = align8(o + 8 * (size_t)(H.num_waves + 1));
        for (int64_t w = 0; w <= H.num_waves; ++w) put_u64(buf + o + 8 * w, voff[w]);
        o = align8(o + 8 * (size_t)(H.num_waves + 1));
        for (int64_t i = 0; i < H.n_words; ++i) put_u32(buf + o + 4 * i, (uint32_t)words.p[i]);
        o = align8(o + 4 * (size_t)H.n_words);
        for (int64_t i = 0; i < H.n_escd; ++i) put_u32(buf + o + 4 * i, (uint32_t)escd.p[i]);
        o = align8(o + 4 * (size_t)H.n_escd);
        for (int64_t i = 0; i < H.n_escv; ++i) {
            if (vsz == 8) put_u64(buf + o + 8 * i, escv.p[i]);
            else put_u32(buf + o + 4 * i, (uint32_t)escv.p[i]);
        }
        o = align8(o + vsz * (size_t)H.n_escv);
        if (sigma) {
            for (int64_t i = 0; i < m; ++i) put_u32(buf + o + 4 * i, (uint32_t)perm[i]);
            o = align8(o + 4 * (size_t)m);
        }
        /* header */
        memcpy(buf, "CSRDTANS", 8);
        put_u32(buf + 8, 1);
        put_u32(buf + 12, H.dtype);
        put_u32(buf + 16, H.layout);
        put_u32(buf + 20, H.lane_nnz);
        put_u64(buf + 24, (uint64_t)H.m);
        put_u64(buf + 32, (uint64_t)H.n);
        put_u64(buf + 40, (uint64_t)H.nnz);
        put_u64(buf + 48, (uint64_t)H.num_lanes);
        put_u64(buf + 56, (uint64_t)H.num_waves);
        put_u64(buf + 64, (uint64_t)H.n_words);
        put_u64(buf + 72, (uint64_t)H.n_escd);
        put_u64(buf + 80, (uint64_t)H.n_escv);
        put_u64(buf + 88, H.seed);
        put_u32(buf + 104, H.first_mode);
        put_u32(buf + 108, H.esc_mode);
        put_u32(buf + 112, H.sigma);
        put_u64(buf + 96, fnv1a64(buf + OK_HEADER, sz - OK_HEADER));
        FILE *fp = fopen(path, "wb");
        if (!fp || fwrite(buf, 1, sz, fp) != sz) rc = ORC_EIO;
        if (fp) fclose(fp);
        free(buf);
    }
    free(words.p); free(escd.p); free(escv.p);
    free(woff); free(doff); free(voff);
    free(dord); free(vord);
    free(first); free(dkey); free(vkey);
    otable_free(&td); otable_free(&tv);
    return rc;
}

/*
 * Row order of a SELL-C-sigma base (Kreutzer et al., SIAM J. Sci. Comput.
 * 2014), the paper's suggested starting point other than CSR (Sec. VII):
 * within each window of sigma consecutive rows, rows by descending number of
 * nonzeros, ties in their original order; perm[r] = original row of encoded
 * row r.  The encoded matrix is the row-permuted one; a wave (C = 64 lanes)
 * then holds rows of similar lengths.  sigma = 0 keeps the CSR order.
 */
static void sigma_order(int64_t m, const int32_t *row_ptr, uint32_t sigma, int32_t *perm)
{
    for (int64_t i = 0; i < m; ++i) perm[i] = (int32_t)i;
    if (!sigma) return;
    for (int64_t w0 = 0; w0 < m; w0 += sigma) {
        int64_t w1 = w0 + (int64_t)sigma < m ? w0 + (int64_t)sigma : m;
        /* insertion sort: stable, plain */
        for (int64_t i = w0 + 1; i < w1; ++i) {
            int32_t r = perm[i];
            int32_t len = row_ptr[r + 1] - row_ptr[r];
            int64_t j = i;
            while (j > w0 && row_ptr[perm[j - 1] + 1] - row_ptr[perm[j - 1]] < len) {
                perm[j] = perm[j - 1];
                --j;
            }
            perm[j] = r;
        }
    }
}

/*
 * Encode a CSR matrix into a container file.  dtype 1: vals are float,
 * dtype 2: vals are double.  layout 1: one row per lane; layout 2: lane_nnz
 * (multiple of 4) nonzeros per lane.  Columns must be sorted within rows.
 * esc_mode: 0 escapes in separate regions, 1 in the word stream.  sigma:
 * 0, or (layout 1 only, a multiple of 64) the window of the row sort above.
 */
int oracle_encode(const char *path, int64_t m, int64_t n, int64_t nnz,
                  const int32_t *row_ptr, const int32_t *col, const void *vals,
                  int dtype, int layout, int lane_nnz, uint64_t seed, int first_mode, int esc_mode,
                  int sigma)
{
    if (sigma == 0)
        return encode_rows(path, m, n, nnz, row_ptr, col, vals, dtype, layout, lane_nnz, seed, first_mode,
                           esc_mode, 0, NULL);
    if (sigma < 0 || sigma % OK_WAVE || layout != 1 || m < 0 || nnz < 0 || (dtype != 1 && dtype != 2) ||
        row_ptr[0] != 0 || row_ptr[m] != nnz)
        return ORC_EINVAL;
    for (int64_t i = 0; i < m; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return ORC_EINVAL;
    size_t vsz = dtype == 2 ? 8 : 4;
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t *rp2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
    int32_t *c2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    uint8_t *v2 = (uint8_t *)malloc(vsz * (size_t)(nnz > 0 ? nnz : 1));
    sigma_order(m, row_ptr, (uint32_t)sigma, perm);
    rp2[0] = 0;
    for (int64_t r = 0; r < m; ++r) {
        int32_t i = perm[r], len = row_ptr[i + 1] - row_ptr[i];
        memcpy(c2 + rp2[r], col + row_ptr[i], sizeof(int32_t) * (size_t)len);
        memcpy(v2 + vsz * (size_t)rp2[r], (const uint8_t *)vals + vsz * (size_t)row_ptr[i], vsz * (size_t)len);
        rp2[r + 1] = rp2[r] + len;
    }
    int rc = encode_rows(path, m, n, nnz, rp2, c2, v2, dtype, layout, lane_nnz, seed, first_mode, esc_mode,
                         (uint32_t)sigma, perm);
    free(perm); free(rp2); free(c2); free(v2);
    return rc;
}

/* ======================================================================
 * decoder (Alg. 3, one lane after another in 64-lane lockstep)
 * ====================================================================== */

typedef struct {
    uint8_t *buf;
    size_t size;
    ohdr H;
    const uint8_t *dtab, *vtab;
    const int32_t *row_ptr;
    const uint64_t *woff, *doff, *voff; /* may be unaligned: read via get_u64 */
    const uint8_t *woff_b, *doff_b, *voff_b, *words_b, *escd_b, *escv_b, *perm_b;
} ofile;

static int read_file(const char *path, ofile *F)
{
    memset(F, 0, sizeof(*F));
    FILE *fp = fopen(path, "rb");
    if (!fp) return ORC_EIO;
    fseek(fp, 0, SEEK_END);
    long len = ftell(fp);
    fseek(fp, 0, SEEK_SET);
    if (len < OK_HEADER) { fclose(fp); return ORC_ECORRUPT; }
    F->buf = (uint8_t *)malloc((size_t)len);
    F->size = (size_t)len;
    if (fread(F->buf, 1, (size_t)len, fp) != (size_t)len) { fclose(fp); return ORC_EIO; }
    fclose(fp);
    const uint8_t *b = F->buf;
    if (memcmp(b, "CSRDTANS", 8) != 0 || get_u32(b + 8) != 1) return ORC_ECORRUPT;
    ohdr *H = &F->H;
    H->dtype = get_u32(b + 12);
    H->layout = get_u32(b + 16);
    H->lane_nnz = get_u32(b + 20);
    H->m = (int64_t)get_u64(b + 24);
    H->n = (int64_t)get_u64(b + 32);
    H->nnz = (int64_t)get_u64(b + 40);
    H->num_lanes = (int64_t)get_u64(b + 48);
    H->num_waves = (int64_t)get_u64(b + 56);
    H->n_words = (int64_t)get_u64(b + 64);
    H->n_escd = (int64_t)get_u64(b + 72);
    H->n_escv = (int64_t)get_u64(b + 80);
    H->seed = get_u64(b + 88);
    H->first_mode = get_u32(b + 104);
    if (H->first_mode > 1) return ORC_ECORRUPT;
    H->esc_mode = get_u32(b + 108);
    if (H->esc_mode > 1 || (H->esc_mode == 1 && (H->n_escd != 0 || H->n_escv != 0))) return ORC_ECORRUPT;
    H->sigma = get_u32(b + 112);
    if (H->sigma % OK_WAVE || (H->sigma && H->layout != 1)) return ORC_ECORRUPT;
    if (fnv1a64(b + OK_HEADER, F->size - OK_HEADER) != get_u64(b + 96)) return ORC_ECORRUPT;
    if ((H->dtype != 1 && H->dtype != 2) || (H->layout != 1 && H->layout != 2)) return ORC_ECORRUPT;
    if (H->m < 0 || H->n < 0 || H->nnz < 0 || H->n_words < 0 || H->n_escd < 0 || H->n_escv < 0)
        return ORC_ECORRUPT;
    size_t vsz = H->dtype == 2 ? 8 : 4;
    size_t o = OK_HEADER;
    size_t need = o;
    need = align8(need + 16 * OK_SLOTS);
    need = align8(need + 16 * OK_SLOTS);
    need = align8(need + 4 * (size_t)(H->m + 1));
    need = align8(need + 3 * align8(8 * (size_t)(H->num_waves + 1)));
    need = align8(need + 4 * (size_t)H->n_words);
    need = align8(need + 4 * (size_t)H->n_escd);
    need = align8(need + vsz * (size_t)H->n_escv);
    if (H->sigma) need = align8(need + 4 * (size_t)H->m);
    if (need != F->size) return ORC_ECORRUPT;
    F->dtab = b + o; o = align8(o + 16 * OK_SLOTS);
    F->vtab = b + o; o = align8(o + 16 * OK_SLOTS);
    F->row_ptr = (const int32_t *)(b + o); o = align8(o + 4 * (size_t)(H->m + 1));
    F->woff_b = b + o; o = align8(o + 8 * (size_t)(H->num_waves + 1));
    F->doff_b = b + o; o = align8(o + 8 * (size_t)(H->num_waves + 1));
    F->voff_b = b + o; o = align8(o + 8 * (size_t)(H->num_waves + 1));
    F->words_b = b + o; o = align8(o + 4 * (size_t)H->n_words);
    F->escd_b = b + o; o = align8(o + 4 * (size_t)H->n_escd);
    F->escv_b = b + o; o = align8(o + vsz * (size_t)H->n_escv);
    F->perm_b = H->sigma ? b + o : NULL;
    /* geometry */
    int64_t lanes = H->layout == 1 ? H->m
                                   : (H->lane_nnz ? (H->nnz + H->lane_nnz - 1) / H->lane_nnz : -1);
    if (H->layout == 2 && (H->lane_nnz == 0 || H->lane_nnz % 4)) return ORC_ECORRUPT;
    if (lanes != H->num_lanes || H->num_waves != (lanes + OK_WAVE - 1) / OK_WAVE) return ORC_ECORRUPT;
    if (F->row_ptr[0] != 0 || F->row_ptr[H->m] != H->nnz) return ORC_ECORRUPT;
    for (int64_t i = 0; i < H->m; ++i)
        if (F->row_ptr[i + 1] < F->row_ptr[i]) return ORC_ECORRUPT;
    return ORC_OK;
}

typedef struct {
    uint64_t sym[OK_SLOTS];
    uint8_t digit[OK_SLOTS];
    uint16_t base[OK_SLOTS];
    uint8_t used[OK_SLOTS], esc[OK_SLOTS];
} dtable;

static int read_table(const uint8_t *b, dtable *t, int is_delta)
{
    for (int i = 0; i < OK_SLOTS; ++i) {
        const uint8_t *e = b + 16 * (size_t)i;
        t->used[i] = e[10] & 1;
        t->esc[i] = (e[10] >> 1) & 1;
        t->sym[i] = get_u64(e);
        t->digit[i] = e[8];
        t->base[i] = (uint16_t)(e[9] + 1);
        if (t->used[i] && t->digit[i] >= t->base[i]) return ORC_ECORRUPT;
        if (t->used[i] && is_delta && !t->esc[i] && t->sym[i] >= OK_DELTA_LIMIT) return ORC_ECORRUPT;
    }
    return ORC_OK;
}

/*
 * Rows of a sigma-sorted container back into their original order (in place
 * on the decoder's outputs).  The stored order must be the one sigma_order
 * gives for the decoded row lengths.
 */
static int unpermute_rows(const ohdr *H, const uint8_t *perm_b, int32_t *row_ptr, int32_t *col, void *vals)
{
    int64_t m = H->m, nnz = H->nnz;
    size_t vsz = H->dtype == 2 ? 8 : 4;
    size_t mm = (size_t)(m > 0 ? m : 1), nn = (size_t)(nnz > 0 ? nnz : 1);
    int32_t *perm = (int32_t *)malloc(4 * mm), *chk = (int32_t *)malloc(4 * mm);
    int32_t *rp = (int32_t *)malloc(4 * (size_t)(m + 1)), *c = (int32_t *)malloc(4 * nn);
    uint8_t *v = (uint8_t *)malloc(vsz * nn), *seen = (uint8_t *)calloc(mm, 1);
    int rc = ORC_OK;
    for (int64_t r = 0; r < m && rc == ORC_OK; ++r) {
        int64_t i = (int32_t)get_u32(perm_b + 4 * r);
        if (i < 0 || i >= m || seen[i] || i / H->sigma != r / H->sigma) rc = ORC_ECORRUPT;
        else { seen[i] = 1; perm[r] = (int32_t)i; }
    }
    if (rc == ORC_OK) {
        for (int64_t r = 0; r < m; ++r) rp[perm[r] + 1] = row_ptr[r + 1] - row_ptr[r];
        rp[0] = 0;
        for (int64_t i = 0; i < m; ++i) rp[i + 1] += rp[i];
        sigma_order(m, rp, H->sigma, chk);
        if (m > 0 && memcmp(chk, perm, 4 * (size_t)m) != 0) rc = ORC_ECORRUPT;
    }
    if (rc == ORC_OK) {
        for (int64_t r = 0; r < m; ++r) {
            int32_t i = perm[r], len = row_ptr[r + 1] - row_ptr[r];
            memcpy(c + rp[i], col + row_ptr[r], 4 * (size_t)len);
            memcpy(v + vsz * (size_t)rp[i], (const uint8_t *)vals + vsz * (size_t)row_ptr[r], vsz * (size_t)len);
        }
        memcpy(row_ptr, rp, 4 * (size_t)(m + 1));
        memcpy(col, c, 4 * (size_t)nnz);
        memcpy(vals, v, vsz * (size_t)nnz);
    }
    free(perm); free(chk); free(rp); free(c); free(v); free(seen);
    return rc;
}

/*
 * Decode a container into CSR arrays (row_ptr: m+1, col: nnz, vals: nnz of
 * the container's dtype), rows in their original order.  Returns 0 or an error code; any inconsistency
 * between the words a decoder consumes and the words stored is an error.
 */
int oracle_decode(const char *path, int32_t *row_ptr_out, int32_t *col_out, void *vals_out)
{
    ofile F;
    int rc = read_file(path, &F);
    if (rc != ORC_OK) { free(F.buf); return rc; }
    const ohdr *H = &F.H;
    static dtable td, tv;
    if (read_table(F.dtab, &td, 1) != ORC_OK || read_table(F.vtab, &tv, 0) != ORC_OK) {
        free(F.buf);
        return ORC_ECORRUPT;
    }
    memcpy(row_ptr_out, F.row_ptr, 4 * (size_t)(H->m + 1));
    uint8_t *first = row_start_flags(H->m, H->nnz, F.row_ptr);
    for (int64_t w = 0; w < H->num_waves && rc == ORC_OK; ++w) {
        uint64_t wp = get_u64(F.woff_b + 8 * w), wend = get_u64(F.woff_b + 8 * (w + 1));
        uint64_t dp = get_u64(F.doff_b + 8 * w), dend = get_u64(F.doff_b + 8 * (w + 1));
        uint64_t vp = get_u64(F.voff_b + 8 * w), vend = get_u64(F.voff_b + 8 * (w + 1));
        if (wend < wp || wend > (uint64_t)H->n_words || dend < dp || dend > (uint64_t)H->n_escd ||
            vend < vp || vend > (uint64_t)H->n_escv) { rc = ORC_ECORRUPT; break; }
        int64_t g0[OK_WAVE], c[OK_WAVE], S[OK_WAVE], maxS = 0;
        uint32_t wd[OK_WAVE][3];
        u128 d[OK_WAVE], r[OK_WAVE];
        uint32_t colv[OK_WAVE];
        for (int q = 0; q < OK_WAVE; ++q) {
            int64_t l = w * OK_WAVE + q;
            g0[q] = 0; c[q] = 0;
            if (l < H->num_lanes) lane_range(H, F.row_ptr, l, &g0[q], &c[q]);
            S[q] = (c[q] + 3) / 4;
            if (S[q] > maxS) maxS = S[q];
            d[q] = 0; r[q] = 1; colv[q] = 0;
        }
#define NEXT_WORD(dst) do { if (wp >= wend) { rc = ORC_ECORRUPT; goto wave_done; } \
        dst = get_u32(F.words_b + 4 * wp); ++wp; } while (0)
        for (int k = 0; k < 3; ++k)
            for (int q = 0; q < OK_WAVE; ++q)
                if (S[q] > 0) NEXT_WORD(wd[q][k]);
        for (int64_t j = 0; j < maxS; ++j) {
            int slot[OK_WAVE][8];
            for (int q = 0; q < OK_WAVE; ++q) {
                if (j >= S[q]) continue;
                unpack8(wd[q], slot[q]);
                for (int t = 0; t < 8; ++t) {
                    const dtable *T = (t % 2 == 0) ? &td : &tv;
                    if (!T->used[slot[q][t]]) { rc = ORC_ECORRUPT; goto wave_done; }
                }
            }
            /* symbols: deltas with escapes, in (position, lane) order */
            for (int pos = 0; pos < 4; ++pos)
                for (int q = 0; q < OK_WAVE; ++q) {
                    int64_t t = 4 * j + pos;
                    if (j >= S[q] || t >= c[q]) continue;
                    int s = slot[q][2 * pos];
                    uint64_t delta;
                    if (td.esc[s] && H->esc_mode == 1) {
                        uint32_t w32;
                        NEXT_WORD(w32);
                        delta = w32;
                    } else if (td.esc[s]) {
                        if (dp >= dend) { rc = ORC_ECORRUPT; goto wave_done; }
                        delta = get_u32(F.escd_b + 4 * dp); ++dp;
                    } else {
                        delta = td.sym[s];
                    }
                    int64_t g = g0[q] + t;
                    uint64_t cc = (t == 0 || first[g])
                                      ? (uint32_t)(first_base(H->first_mode, row_of(F.row_ptr, H->m, g)) +
                                                   (uint32_t)delta)
                                      : (uint64_t)colv[q] + delta;
                    if (cc >= (uint64_t)H->n) { rc = ORC_ECORRUPT; goto wave_done; }
                    colv[q] = (uint32_t)cc;
                    col_out[g] = (int32_t)cc;
                }
            for (int pos = 0; pos < 4; ++pos)
                for (int q = 0; q < OK_WAVE; ++q) {
                    int64_t t = 4 * j + pos;
                    if (j >= S[q] || t >= c[q]) continue;
                    int s = slot[q][2 * pos + 1];
                    uint64_t bits;
                    if (tv.esc[s] && H->esc_mode == 1) {
                        uint32_t lo, hi = 0;
                        NEXT_WORD(lo);
                        if (H->dtype == 2) NEXT_WORD(hi);
                        bits = (uint64_t)hi << 32 | lo;
                    } else if (tv.esc[s]) {
                        if (vp >= vend) { rc = ORC_ECORRUPT; goto wave_done; }
                        bits = H->dtype == 2 ? get_u64(F.escv_b + 8 * vp) : get_u32(F.escv_b + 4 * vp);
                        ++vp;
                    } else {
                        bits = tv.sym[s];
                    }
                    int64_t g = g0[q] + t;
                    if (H->dtype == 2) memcpy((double *)vals_out + g, &bits, 8);
                    else { uint32_t b32 = (uint32_t)bits; memcpy((float *)vals_out + g, &b32, 4); }
                }
            /* state: group g appends its 4 digits, then check g, lane order */
            for (int g = 0; g < 2; ++g)
                for (int q = 0; q < OK_WAVE; ++q) {
                    if (j >= S[q] - 1) continue; /* last segment: no checks */
                    for (int t = 4 * g; t < 4 * g + 4; ++t) {
                        const dtable *T = (t % 2 == 0) ? &td : &tv;
                        int s = slot[q][t];
                        d[q] = d[q] * T->base[s] + T->digit[s];
                        r[q] = r[q] * T->base[s];
                    }
                    if (r[q] >= ((u128)1 << 32)) {
                        wd[q][g] = (uint32_t)(d[q] & 0xffffffffu);
                        d[q] >>= 32;
                        r[q] >>= 32;
                    } else {
                        NEXT_WORD(wd[q][g]);
                    }
                }
            for (int q = 0; q < OK_WAVE; ++q)
                if (j < S[q] - 1) NEXT_WORD(wd[q][2]);
        }
        if (wp != wend || dp != dend || vp != vend) rc = ORC_ECORRUPT;
    wave_done:;
#undef NEXT_WORD
    }
    if (rc == ORC_OK && H->sigma) rc = unpermute_rows(H, F.perm_b, row_ptr_out, col_out, vals_out);
    free(first);
    free(F.buf);
    return rc;
}

/* header fields: out[0..15] = dtype, layout, lane_nnz, m, n, nnz, num_lanes,
 * num_waves, n_words, n_escd, n_escv, seed, file size, first-delta mode,
 * escape mode, row-sort window */
int oracle_read_header(const char *path, int64_t *out)
{
    ofile F;
    int rc = read_file(path, &F);
    if (rc == ORC_OK) {
        out[0] = F.H.dtype; out[1] = F.H.layout; out[2] = F.H.lane_nnz;
        out[3] = F.H.m; out[4] = F.H.n; out[5] = F.H.nnz;
        out[6] = F.H.num_lanes; out[7] = F.H.num_waves; out[8] = F.H.n_words;
        out[9] = F.H.n_escd; out[10] = F.H.n_escv; out[11] = (int64_t)F.H.seed;
        out[12] = (int64_t)F.size; out[13] = F.H.first_mode; out[14] = F.H.esc_mode;
        out[15] = F.H.sigma;
    }
    free(F.buf);
    return rc;
}
