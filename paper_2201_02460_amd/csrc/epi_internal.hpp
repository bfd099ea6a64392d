// Internal layout shared by the host runtime and the gfx950 kernels.
//
// Device layout of a packed dataset (the genotype tables of Section 2.1 of the
// paper, stored per class and per genotype as bitsets of individuals):
//
//   masks   : v4u [(W4[0] + W4[1]) * 2][Mp]
//             element ((wbase[c] + w4) * 2 + g) * Mp + s holds bits
//             128*w4 .. 128*w4+127 of class c's row for genotype g of SNP s
//             (4 x 32-bit words, bit b of word q = individual 32*(4*w4+q)+b
//             of that class, in input order).  Only genotypes 0 and 1 are
//             stored; genotype 2 is valid & ~(row0 | row1).  Bits past the
//             class size and SNPs s >= M are zero.  Class 0 = cases.
//   single  : u32 [Mp][2 classes][2 genotypes] per-SNP class counts of
//             genotypes 0 and 1.
//   tlog    : i64 [2N + 1], tlog[n] = round(n * ln(n) * 2^shift).
//   itab    : u32 [2N + 2], t(n) = round(n * ln(n) * 2^tq) mod 2^32 at entries
//             n = 0 .. N and again at entries 2N + 1 - n (the screening table;
//             copied to LDS address 0, t(n) is at byte 4n and at byte
//             q3_bias(N) - 4n).
//   qa, qb  : the same genotype-0/1 rows as 4-bit floats (e2m1: qa 0x2 = 1.0,
//             qb 0x6 = 4.0, 0x0 = 0), in the operand order of the 32x32x64 matrix-core
//             product: one 16-byte entry per lane = 32 individuals of one row.
//             KS = ks[0] + ks[1] steps of 64 individuals (class 0 first, each
//             class zero-padded to a multiple of kQStepMultiple steps); half h
//             of a step holds its
//             individuals 32h .. 32h+31, two per byte, low nibble first.
//             qa [((s / 16) * KS + step) * 64 + 32 h + 2 (s % 16) + g]
//             qb [(((s / 32) * 2 + g) * KS + step) * 64 + 32 h + s % 32]
//   qa8, qb8: the same with 8-bit integer operands (qa8 1, qb8 4) for the
//             32x32x32 integer product: steps of 32 individuals (ks8 per
//             class, padded alike), half h = individuals 16h .. 16h+15, one
//             per byte; built only when the integer kernel is selected.
//
// Lanes of a wave read 16 consecutive bytes each of 64 consecutive SNPs, so a
// wave-wide load of one mask row group is one contiguous 1 KiB segment.
#pragma once

#include <stdint.h>

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

namespace epi {

constexpr int kMaxTopK = 256;
// Entries of a wave's best-K list in LDS for a best-K of top_k: room for a
// wave's worth of new candidates past K, a power of two (the list is sorted
// in place when a batch of candidates overflows it).
__host__ __device__ constexpr int list_cap(int top_k) {
    int c = 64;
    while (c < top_k + 64) c <<= 1;
    return c;
}
constexpr int kWave = 64;
constexpr int kMergeSlots = 4096;      // LDS entries of the top-K merge
constexpr int kMergeParts = 32;        // first-stage merge workgroups per task
constexpr int kMaxBinomOrder = 8;
constexpr int kNpMfma = 16;            // order-3 block counted by matrix cores, 4-bit float operands
constexpr int kNpMfmaI8 = 32;          // the same with 8-bit integer operands
constexpr int kNpMfma2 = 48;           // 4-bit float operands, two middle SNPs per work item, both
                                       // classes in one accumulator

// Prefix blocks of the matrix-core order-3 kernels (their work items and
// signed cell form differ from the popcount kernels').
__host__ __device__ constexpr bool is_mfma_np(int np) { return np == kNpMfma || np == kNpMfmaI8 || np == kNpMfma2; }
constexpr int kQStepMultiple = 4;      // qa / qb: steps per class padded to a multiple of this

// The two-middle-SNP matrix-core kernel scales the control steps' products by
// 2^(T - 2) (the MFMA's per-block exponent scale), so one float accumulator
// holds 4 n(cases) + 2^T n(controls) with T = 2 + bit width of the case
// count: the cases' field is below 2^T and the sum stays an exact float
// integer while it is below 2^24.
__host__ __device__ inline int q3_pack_shift(int n_cases) {
    return n_cases <= 0 ? 2 : 34 - __builtin_clz((unsigned)n_cases);
}
__host__ __device__ inline bool q3_pack_fits(int n_cases, int n_controls) {
    const int T = q3_pack_shift(n_cases);
    return n_cases >= 0 && n_controls >= 0 && T <= 24 &&
           4ull * (unsigned long long)n_cases + ((unsigned long long)n_controls << T) < (1ull << 24);
}
constexpr int kQStageSteps = 64;       // matrix-core kernels: steps of j-mask rows staged in LDS

enum Variant : int32_t {
    kGeneric = 0,  // one combination per lane, all 3^k cells counted
    kF2 = 1,       // order 2, reduced cells, prefix block of i's
    kF3 = 2,       // order 3, reduced cells, prefix block of i's sharing j
    kF2Emit = 3,   // order-2 reduced cells written to the pair sub-table
    kF3Emit = 4,   // order-3 reduced cells written to the triplet sub-table (matrix cores)
    kR4 = 5,       // order 4, reduced cells per lane, other cells from the sub-tables
    kSeg = 6,      // any order, segmented: a wave's 64 tables counted to a buffer, then scored
    kF2Fold = 7,   // order 2 scored by the pair sub-table pass of another scan of the same dataset
};

// Kernel instantiation of the segmented variant for order k: generic-order
// parameter kSegGk + k.
constexpr int kSegGk = 16;

struct DsView {
    const v4u *masks;
    const uint32_t *single;
    const long long *tlog;
    const uint32_t *itab;  // screening table: t(n) = round(n ln n 2^tq) mod 2^32 for
                           // n = 0 .. N, then the same values for n = N .. 0
    const v4u *qa, *qb;    // 4-bit-float operand copies of the masks
    const v4u *qa8, *qb8;  // 8-bit-integer operand copies (null until selected)
    int32_t tq;            // fixed-point scale of itab (2^tq per unit of n ln n)
    int32_t M, Mp, N, shift;
    int32_t ncls[2];
    int32_t w4[2];
    int32_t wbase[2];
    int32_t ks[2];         // 64-individual steps per class in qa / qb
    int32_t ks8[2];        // 32-individual steps per class in qa8 / qb8
    const int *err;        // error bits of the dataset's last packing (0: valid input)
};

// One top-K candidate: larger num is better; on equal num the smaller key
// (the combination's indices packed big-endian) is better.
struct Cand {
    long long num;
    unsigned long long key;
};

struct Task {
    DsView ds;
    uint32_t *pairs;                  // pair sub-table, 8 u32 per pair (lexicographic, or colex: pair_colex)
    uint32_t *triples;                // colex-ordered triplet sub-table, 8 u32 per triplet (kR4, kF3Emit)
    uint32_t *seg;                    // kSeg: per wave slot of the launch (4 per workgroup), 2 x 3^k x 64 u32
                                      //   counts, cell-major ([class][cell][lane])
    const unsigned long long *items;  // per-item descriptors: kF3 j<<40 | ib<<20 | mb, kF2 ib<<20 | mb
                                      // (kF3 with np = kNpMfma: 16-SNP i-block ib, 32-SNP m-block mb)
    unsigned long long n_items;
    unsigned long long item_base;     // first global item of this task in its launch
    unsigned long long first_item;    // task-local index of the launch's first item of this task
    unsigned long long n_combos;
    long long score_const;            // tlog[N] - tlog[n_case] - tlog[n_ctrl]
    Cand *cand;                       // candidate sink
    unsigned int *cand_count;
    unsigned long long *thr;          // running lower bound of the K-th best num (sign-flipped int64)
    unsigned int *hist;               // score histogram, kHistWords counters (null: none)
    unsigned int cand_cap;
    int32_t variant, order, top_k;
    int32_t np;                       // prefix block (kF2/kF3) or ranks per lane (kGeneric)
    int32_t n_blocks;                 // number of prefix blocks (kF2: i-blocks, kF3: j values + 1)
    int32_t key_bits;                 // bits per index in the packed key
    int32_t cell_shift;               // kF2Emit: pair cells are written as (count << cell_shift)
    uint32_t cell_bias;               //   + cell_bias, or with cell_neg as cell_bias - (count << cell_shift)
    int32_t cell_neg;
    int32_t pair_colex;               // kF2Emit: pair rows at colex ranks C(m,2) + i, one word per cell
                                      //   with both classes (the reduced order-4 kernel's lanes vary the
                                      //   lowest index), else lexicographic
    unsigned long long *digest;       // checking launches: [0] combinations scored, [1] their digest sum
                                      //   (null: no check)
    unsigned long long pilot_first;   // matrix-core order 3, order 4 by reduced cells: items
    int32_t pilot_n;                  //   pilot_first .. + pilot_n - 1 were counted into the histogram by
                                      //   the pilot pass (0: none; a multiple of 4)
    unsigned long long pilot_base;    // the task's first item in its pilot launch (a multiple of 4)
};

// Work-item descriptor tables, one item per entry, in groups of consecutive
// items (the layouts the kernels decode, see Task::items):
//   kItemsF2   order 2, prefix block np: group ib (block of np first SNPs),
//              items ib << 20 | mb for the ceil(max(0, M - 1 - ib np) / 64)
//              blocks mb of 64 last SNPs;
//   kItemsF3   order 3 by popcount, prefix block np: group j = 1 .. M - 2,
//              items j << 40 | ib << 20 | mb for ib < ceil(j / np) (outer)
//              and mb < ceil((M - 1 - j) / 64) (inner);
//   kItemsF3M  order 3 by matrix cores: group (block ib of 16 first SNPs,
//              block mb of 32 last SNPs), items j << 40 | ib << 20 | mb for
//              every j with some i < j < m in the blocks, j fastest.  The
//              groups go in tiles of 4 x 4 blocks (tile rows of mb outer,
//              then tiles of ib; mb outer, ib inner within a tile), so the
//              items in flight across the device share a few operand blocks;
//   kItemsF3M2 the same groups, one item per two consecutive middle SNPs j,
//              j + 1 (descriptor of the first; the last item of an odd run
//              has one);
//   kItemsF2M  order 2 by matrix cores: group ib (block of 32 first SNPs
//              i0 = 32 ib), items ib << 20 | mb for the blocks mb of 32 last
//              SNPs (m = 32 mb ..) from the one holding i0 + 1 on.
// The host counts a table's items with these functions and the device
// writes them (items_kernel), group after group.
enum ItemKind : int32_t { kItemsF2 = 0, kItemsF3 = 1, kItemsF3M = 2, kItemsF3M2 = 3, kItemsF2M = 4 };
constexpr int kItemTile = 4;
constexpr int kStoreChunkBytes = 1024;  // bytes per store_kernel launch

struct ItemGroup {
    unsigned long long base;  // descriptor of the group's first item
    unsigned long long step;  // added per item (kItemsF3: per item of the inner run)
    unsigned long long count; // items in the group
    unsigned long long inner; // kItemsF3: items per ib (0: one run)
};

__host__ __device__ inline long long item_groups(int kind, int M, int np) {
    if (kind == kItemsF2) return M >= 2 ? (M - 1 + np - 1) / np : 0;
    if (kind == kItemsF3) return M >= 3 ? M - 2 : 0;
    if (kind == kItemsF2M) return M >= 2 ? (M + 31) / 32 : 0;
    return (long long)((M + 31) / 32) * ((M + 15) / 16);
}

__host__ __device__ inline ItemGroup item_group(int kind, int M, int np, long long g) {
    ItemGroup r{0, 1, 0, 0};
    if (kind == kItemsF2) {
        const long long ib = g, nm = M - 1 - ib * np;
        r.base = (unsigned long long)ib << 20;
        r.count = nm > 0 ? (unsigned long long)((nm + 63) / 64) : 0;
        return r;
    }
    if (kind == kItemsF2M) {
        const long long i0 = g * 32, mb0 = (i0 + 1) / 32, nmb = (M + 31) / 32;
        r.base = ((unsigned long long)g << 20) | (unsigned long long)mb0;
        r.count = i0 + 1 < M ? (unsigned long long)(nmb - mb0) : 0;
        return r;
    }
    if (kind == kItemsF3) {
        const long long j = g + 1, ni = (j + np - 1) / np, nm = (M - 1 - j + 63) / 64;
        r.base = (unsigned long long)j << 40;
        r.inner = (unsigned long long)nm;
        r.count = (unsigned long long)(ni * nm);
        return r;
    }
    const long long nmb = (M + 31) / 32, nib = (M + 15) / 16, T = kItemTile;
    const long long mt = g / (T * nib), rr = g - mt * T * nib;
    const long long mbs = nmb - mt * T < T ? nmb - mt * T : T;
    const long long it = rr / (mbs * T), q = rr - it * mbs * T;
    const long long ibs = nib - it * T < T ? nib - it * T : T;
    const long long mb = mt * T + q / ibs, ib = it * T + q % ibs;
    long long j0 = ib * 16 + 1, j1 = (mb * 32 + 31 < M - 1 ? mb * 32 + 31 : M - 1) - 1;
    j0 = j0 > 1 ? j0 : 1;
    j1 = j1 < M - 2 ? j1 : M - 2;
    r.base = ((unsigned long long)j0 << 40) | ((unsigned long long)ib << 20) | (unsigned long long)mb;
    const unsigned long long run = j1 >= j0 ? (unsigned long long)(j1 - j0 + 1) : 0;
    r.step = (kind == kItemsF3M2 ? 2ull : 1ull) << 40;
    r.count = kind == kItemsF3M2 ? (run + 1) / 2 : run;
    return r;
}

// Descriptor of item t of a group.
__host__ __device__ inline unsigned long long item_at(const ItemGroup &gr, unsigned long long t) {
    if (gr.inner) return gr.base + ((t / gr.inner) << 20) + t % gr.inner;
    return gr.base + t * gr.step;
}

// Completeness check of a scan (every combination exactly once, each with
// its table).  mix64 is the output function of SplitMix64 (Steele, Lea and
// Flood, "Fast splittable pseudorandom number generators", 2014).  A
// combination c_1 < ... < c_k with table T[class][x] (class 0 = cases, x the
// cell index) contributes mix64(h ^ s), where h folds its indices,
// h = mix64(... mix64(mix64(c_1 + 1) + c_2 + 1) ... + c_k + 1), and s weighs
// its counts, s = sum T[class][x] * mix64(2 x + class + 1) (all mod 2^64).
// A scan's digest is the sum of the contributions of the combinations it
// scored, so it does not depend on the order in which they were visited.
__host__ __device__ constexpr unsigned long long mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__host__ __device__ constexpr unsigned long long cell_weight(int cls, int x) {
    return mix64(2ull * (unsigned long long)x + (unsigned long long)cls + 1ull);
}

// Score histogram of a task: how many distinct combinations entered some
// wave's best-K list (or, pilot items, lower bounds of their best scores), by
// the position of the leading bit of their num and the next kHistFineBits
// bits (64 x 2^kHistFineBits counters).  It turns the lists of all waves
// into one lower bound of the task's K-th best.  A positive num has its
// leading bit at position 62 at most, so the bins of position 63 are never
// counted; the last word is the task's pilot counter instead.
constexpr int kHistFineBits = 5;
constexpr int kHistFine = 1 << kHistFineBits;
constexpr int kHistWords = 64 * kHistFine;
constexpr int kHistTop = 63 * kHistFine - 1;  // highest bin a positive num reaches
constexpr int kPilotWord = kHistWords - 1;    // pilot items of the task done so far

// Matrix-core order-3 kernels count 4 x n (their B operand holds 4 for a set
// bit), so a count is also the byte offset of its screening-table entry.
// Their epilogue holds a cell with an odd number of marginal SNPs as
// q3_bias(N) - 4n and the others as 4n, and takes its marginal inputs with
// offsets that keep that form through the inclusion-exclusion (a multiple
// o_t of q3_bias(N) for t marginal SNPs: 1, -4, 13 for t = 1 .. 3, sign
// (-1)^t on the 4n).  So their pair sub-table is written with cell_shift =
// kQScaleShift, cell_bias = q3_bias(N), cell_neg = 1.  Order 4 by reduced
// cells holds both classes of a cell in one word instead, 4 n(cases) |
// 4 n(controls) << 16 (pair_colex pair sub-table, 16 B per pair; triplet
// sub-table 32 B per triplet).
constexpr int kQScaleShift = 2;

// Byte offset just past the screening table's two halves (2N + 2 entries):
// t(n) of the second half sits at q3_bias(N) - 4 n.
constexpr uint32_t q3_bias(int N) { return 8u * (uint32_t)N + 4u; }

// Per-task result block written by the finalize kernel:
//   int32 n_valid, int32 pack_err (the dataset's packing error bits when the
//   block was written), int32 pad[2],
//   int32 combos[top_k][order], float scores[top_k],
//   uint32 tables[top_k][2][3^order]
struct ResultLayout {
    long long offset;  // byte offset of the block in the plan's result buffer
    int32_t top_k, order;
};

inline int pow3i(int k) {
    int p = 1;
    for (int t = 0; t < k; ++t) p *= 3;
    return p;
}

inline long long result_block_bytes(int top_k, int order) {
    long long b = 16 + (long long)top_k * order * 4 + (long long)top_k * 4 +
                  (long long)top_k * 2 * pow3i(order) * 4;
    return (b + 255) & ~255LL;
}

}  // namespace epi
