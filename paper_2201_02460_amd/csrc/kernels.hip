// gfx950 kernels of the exhaustive k-order epistasis scan.
//
// Paper mapping:
//   pack_kernel / singles_kernel  genotype tables of single SNPs (Section 2.1)
//   scan_persistent               enumeration (Algorithm 1), contingency
//                                 tables (Section 2.2), mutual information
//                                 (Section 2.3, Equations 1-3), best-K
//                                 retention (Section 2.4)
//   merge_part/final_kernel       final best-K selection (two stages)
//   finalize_kernel               combinations, scores and full 2 x 3^k
//                                 tables of the retained combinations
//
// Counting.  The paper intersects genotype rows with AND and counts bits.  A
// cell of a combination's table is popcount(AND of one row per SNP).  Here a
// lane counts the cells of one combination; the rows of SNPs shared by every
// lane of the wave (the prefix of Algorithm 1) are staged once per work item
// in the wave's LDS slot and read back with broadcast loads, so each cell of
// each 32-individual word costs one v_bitop3_b32 (three-input AND) and one
// v_bcnt_u32_b32 (popcount + accumulate).
//
// Reduced cells (kF2, kF3).  Only cells whose genotypes are all 0 or 1 are
// counted.  Every other cell follows exactly by inclusion-exclusion from
// counts of sub-combinations: the indicator of genotype 2 is 1 minus the
// indicators of genotypes 0 and 1, so a cell with genotype 2 at SNP t equals
// the table of the combination without SNP t minus the two cells with
// genotype 0 and 1 at t.  Order 2 needs the single-SNP counts, order 3 the
// pair sub-table (written by the kF2Emit variant) as well.  The integers are
// those of counting all 3^k cells.
//
// Score.  N * MI = sum_xy n_xy ln n_xy - sum_x n_x ln n_x - sum_y n_y ln n_y
// + N ln N (Equation 1 with p = n / N).  Each n ln n is read from a table of
// round(n ln n * 2^shift) and summed in int64, so the score of a combination
// is the same integer whatever kernel, tile or batch computes it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <type_traits>

#include "epi_internal.hpp"

namespace epi {

typedef __attribute__((address_space(4))) const v4u cv4u;  // wave-uniform rows: scalar loads
typedef __attribute__((address_space(1))) const v4u gv4u;  // per-lane rows: vector loads

#define EPI_DEV __device__ __forceinline__

// popcount(x) + acc as one v_bcnt_u32_b32 (the compiler would otherwise
// reassociate chains of popcounts into extra v_add3 instructions).
EPI_DEV unsigned bcnt_acc(unsigned x, unsigned acc) {
    unsigned r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// a + b + c as one v_add3_u32 (the compiler splits sums with a subtracted
// term into two-operand adds and subtracts).
EPI_DEV unsigned add3(unsigned a, unsigned b, unsigned c) {
    unsigned r;
    asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

EPI_DEV unsigned long long rfl64(unsigned long long v) {
    unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

EPI_DEV unsigned long long readlane64(unsigned long long v, int lane) {
    unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, lane);
    unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), lane);
    return ((unsigned long long)hi << 32) | lo;
}

EPI_DEV int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Orders this wave's LDS accesses (lane-0 writes before all-lane reads) without
// a workgroup barrier: the waves of a workgroup run independently.
EPI_DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

EPI_DEV unsigned lane_prefix(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Pin a wave-uniform value to a scalar register (values decoded with VALU
// arithmetic, such as integer division, would otherwise stay in VGPRs and
// turn the uniform mask-row loads into vector loads).
EPI_DEV int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

EPI_DEV unsigned long long bias(long long v) { return (unsigned long long)v ^ 0x8000000000000000ull; }
EPI_DEV long long unbias(unsigned long long v) { return (long long)(v ^ 0x8000000000000000ull); }

EPI_DEV long long load_thr(unsigned long long *p) {
    return unbias(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

EPI_DEV bool better(long long an, unsigned long long ak, long long bn, unsigned long long bk) {
    return an > bn || (an == bn && ak < bk);
}

// ---------------------------------------------------------------------------
// Score histogram (layout in epi_internal.hpp).  A combination whose exact num
// enters a wave's list is counted once, in the bin of its leading bit and the
// next kHistFineBits bits; a bin's lower edge is at most the num of everything
// counted in it.  Each combination is scored by one wave only, so K counts at
// or above an edge are K distinct combinations at least that good: nothing
// below the edge can be in the best K.  Counts read while other waves add to
// them are never above the true ones, and leaving bins out only lowers a sum,
// so a bound taken from any part of the histogram is valid.
// ---------------------------------------------------------------------------
EPI_DEV int hist_bin(long long num) {  // num > 0
    const unsigned long long v = (unsigned long long)num;
    const int e = 63 - __builtin_clzll(v);
    const unsigned f = e >= kHistFineBits ? (unsigned)(v >> (e - kHistFineBits)) : (unsigned)(v << (kHistFineBits - e));
    return e * kHistFine + (int)(f & (kHistFine - 1));
}

EPI_DEV long long hist_edge(int bin) {
    const int e = bin / kHistFine;
    const unsigned long long top = (unsigned long long)(kHistFine + bin % kHistFine);
    return (long long)(e >= kHistFineBits ? top << (e - kHistFineBits) : top >> (kHistFineBits - e));
}

EPI_DEV unsigned wave_scan_incl(unsigned v) {
    const int lane = lane_id();
    #pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const unsigned o = __shfl_up(v, off);
        if (lane >= off) v += o;
    }
    return v;
}

// Largest lower edge with at least K counted combinations at or above it, or
// INT64_MIN.  The sum starts one leading-bit position above `top` (the
// highest bin this wave has counted) and runs down over at most two windows
// of 64 bins: a few round trips, however the scores are scaled.
EPI_DEV long long hist_bound(const unsigned *h, int K, int top) {
    const int lane = lane_id();
    int start = top + kHistFine;
    start = start < kHistTop ? start : kHistTop;
    unsigned carry = 0;
    #pragma unroll 1
    for (int w = 0; w < 2; ++w, start -= kWave) {
        const int b = start - lane;
        const unsigned c = b >= 0 ? __hip_atomic_load(h + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        const unsigned cs = wave_scan_incl(c) + carry;
        const unsigned long long m = __ballot(cs >= (unsigned)K);
        if (m) return hist_edge(start - (int)__builtin_ctzll(m));
        carry = (unsigned)__builtin_amdgcn_readlane((int)cs, kWave - 1);
        if (start < kWave) break;
    }
    return (long long)0x8000000000000000ull;
}

// Rank of pair (x, y), x < y, in the lexicographic order of the pairs of M.
EPI_DEV unsigned long long lexpair(long long x, long long y, long long M) {
    return (unsigned long long)(x * (2 * M - x - 1) / 2 + (y - x - 1));
}

// Rank of pair (x, x + 1): x (2M - x - 1) / 2.  Both factors stay below 2^24
// (M < 2^23), which lets the product use the 24-bit multipliers.
EPI_DEV unsigned long long pair_row(int x, int M) {
    const unsigned a = (unsigned)x & 0xffffffu, b = (unsigned)(2 * M - x - 1) & 0xffffffu;
    return ((unsigned long long)a * (unsigned long long)b) >> 1;
}

// Valid-individual bits of words 4*w4 .. 4*w4+3 of a class of n individuals.
EPI_DEV v4u valid_mask(int n, int w4) {
    v4u v;
    #pragma unroll
    for (int q = 0; q < 4; ++q) {
        int left = n - 32 * (4 * w4 + q);
        v[q] = left >= 32 ? 0xffffffffu : (left <= 0 ? 0u : ((1u << left) - 1u));
    }
    return v;
}

// In-place inclusion-exclusion over a 3^2 / 3^3 table whose index 2 along an
// axis holds the marginal over that SNP on input and genotype 2 on output.
EPI_DEV void mobius2(int (&R)[9]) {
    #pragma unroll
    for (int e = 0; e < 3; ++e) R[6 + e] -= R[e] + R[3 + e];
    #pragma unroll
    for (int a = 0; a < 3; ++a) R[3 * a + 2] -= R[3 * a] + R[3 * a + 1];
}

EPI_DEV void mobius3(int (&R)[27]) {
    #pragma unroll
    for (int r = 0; r < 9; ++r) R[18 + r] -= R[r] + R[9 + r];
    #pragma unroll
    for (int a = 0; a < 3; ++a)
        #pragma unroll
        for (int e = 0; e < 3; ++e) R[9 * a + 6 + e] -= R[9 * a + e] + R[9 * a + 3 + e];
    #pragma unroll
    for (int ab = 0; ab < 9; ++ab) R[3 * ab + 2] -= R[3 * ab] + R[3 * ab + 1];
}

template <class T>
EPI_DEV void mobius4(T (&R)[81]) {
    #pragma unroll
    for (int st = 27; st >= 1; st /= 3)
        #pragma unroll
        for (int x = 0; x < 81; ++x)
            if ((x / st) % 3 == 2) R[x] -= R[x - 2 * st] + R[x - st];
}

// Cells whose base-3 index has an odd number of digits 2, held as B - 4n in
// the signed cell form.
constexpr bool odd_twos(int x) { return x == 0 ? false : ((x % 3 == 2) != odd_twos(x / 3)); }

// mobius3 on the signed cell form (B - 4n for odd_twos cells, 4n for the
// others, each marginal input offset so that the result comes out in that
// form): a genotype-2 cell is its marginal minus the genotype-0 and -1 cells,
// which the form turns into one sum of three.
EPI_DEV void mobius3_signed(unsigned (&R)[27]) {
    #pragma unroll
    for (int r = 0; r < 9; ++r) R[18 + r] += R[r] + R[9 + r];
    #pragma unroll
    for (int a = 0; a < 3; ++a)
        #pragma unroll
        for (int e = 0; e < 3; ++e) R[9 * a + 6 + e] += R[9 * a + e] + R[9 * a + 3 + e];
    #pragma unroll
    for (int ab = 0; ab < 9; ++ab) R[3 * ab + 2] += R[3 * ab] + R[3 * ab + 1];
}


// Sub-table passes keep no best-K list.
EPI_DEV bool is_emit(int variant) { return variant == kF2Emit || variant == kF3Emit; }

// Colex rank of x < y: C(y,2) + x.
EPI_DEV unsigned long long colex2(int x, int y) {
    const unsigned long long Y = (unsigned long long)y;
    return Y * (Y - 1) / 2 + (unsigned long long)x;
}

// Colex rank of x < y < z: C(z,3) + C(y,2) + x (z < 2^21).
EPI_DEV unsigned long long colex3(int x, int y, int z) {
    const unsigned long long Z = (unsigned long long)z, Y = (unsigned long long)y;
    return Z * (Z - 1) * (Z - 2) / 6 + Y * (Y - 1) / 2 + (unsigned long long)x;
}

// ---------------------------------------------------------------------------
// Per-wave best-K list in LDS (unsorted) with its current worst entry.
// ---------------------------------------------------------------------------
struct TopK {
    int n, K, wi;
    int cap;         // entries of the list in LDS (list_cap of the launch's largest K)
    long long wn;
    unsigned long long wk;
    unsigned *hist;  // the task's score histogram (null: none)
    int added;       // combinations counted since the bound was last taken
    int top;         // highest histogram bin this wave has counted (-1: none)
    unsigned long long dsum;  // checking launches: this lane's digest sum and count since the last flush
    unsigned dn;
    int nohist;      // the item's combinations are already in the histogram (a pilot item)
};

// ---------------------------------------------------------------------------
// Completeness check (checking launches only; definition in
// epi_internal.hpp): every scored combination adds mix64(h ^ s) to its
// lane's sum, flushed to the task's two counters when the wave leaves the
// task.
// ---------------------------------------------------------------------------
template <int K>
EPI_DEV unsigned long long combo_hash(const int (&c)[K]) {
    unsigned long long h = 0;
    #pragma unroll
    for (int t = 0; t < K; ++t) h = mix64(h + (unsigned long long)c[t] + 1ull);
    return h;
}

EPI_DEV void digest_add(TopK &t, bool valid, unsigned long long h, unsigned long long s) {
    if (valid) {
        t.dsum += mix64(h ^ s);
        t.dn += 1;
    }
}

// Weighted sum of a table held as plain counts F[class][x].
template <int CELLS, class T>
EPI_DEV unsigned long long table_sum(const T (&F0)[CELLS], const T (&F1)[CELLS]) {
    unsigned long long s = 0;
    #pragma unroll
    for (int x = 0; x < CELLS; ++x)
        s += (unsigned long long)(unsigned)F0[x] * cell_weight(0, x) + (unsigned long long)(unsigned)F1[x] * cell_weight(1, x);
    return s;
}

EPI_DEV void digest_flush(TopK &t, const Task &task) {
    unsigned long long s = t.dsum, n = t.dn;
    #pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off);
        n += __shfl_xor(n, off);
    }
    if (lane_id() == 0 && task.digest) {
        atomicAdd(task.digest, n);
        atomicAdd(task.digest + 1, s);
    }
    t.dsum = 0;
    t.dn = 0;
}

// Count the combinations of the lanes with `counted` set: one atomic per
// distinct bin of the wave, with the number of its lanes in that bin.
EPI_DEV void hist_add(TopK &t, bool counted, long long num) {
    counted = counted && num > 0;
    unsigned long long pend = __ballot(counted);
    if (!pend) return;
    const int b = counted ? hist_bin(num) : -1;
    t.added = 1;
    while (pend) {
        const int src = (int)__builtin_ctzll(pend);
        const int bs = __builtin_amdgcn_readlane(b, src);
        const unsigned long long same = pend & __ballot(b == bs);
        if (lane_id() == src)
            __hip_atomic_fetch_add(t.hist + bs, (unsigned)__popcll(same), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t.top = bs > t.top ? bs : t.top;
        pend &= ~same;
    }
}

EPI_DEV void tk_recompute(TopK &t, const Cand *list) {
    const int lane = lane_id();
    long long bn = 0;
    unsigned long long bk = 0;
    int bi = -1;
    for (int i = lane; i < t.n; i += kWave) {
        Cand c = list[i];
        if (bi < 0 || better(bn, bk, c.num, c.key)) {
            bn = c.num;
            bk = c.key;
            bi = i;
        }
    }
    #pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        long long on = __shfl_xor(bn, off);
        unsigned long long ok = __shfl_xor(bk, off);
        int oi = __shfl_xor(bi, off);
        if (oi >= 0 && (bi < 0 || better(bn, bk, on, ok))) {
            bn = on;
            bk = ok;
            bi = oi;
        }
    }
    t.wn = (long long)rfl64((unsigned long long)bn);
    t.wk = rfl64(bk);
    t.wi = __builtin_amdgcn_readfirstlane(bi);
}

// Power of two a list of n entries is sorted in (at least 64).
EPI_DEV int tk_sort_size(int n) {
    int P = 64;
    while (P < n) P <<= 1;
    return P;
}

// Sort the first n entries of a wave's list best first, in place (entries
// n .. P - 1, P = tk_sort_size(n), hold the worst value meanwhile: the
// caller makes sure the list has P entries).  Bitonic network, each lane a
// pair per compare-exchange step.
EPI_DEV void tk_sort(Cand *a, int n) {
    const int P = tk_sort_size(n);
    for (int i = n + lane_id(); i < P; i += kWave) a[i] = Cand{(long long)0x8000000000000000ull, ~0ull};
    wave_sync();
    #pragma unroll 1
    for (int k = 2; k <= P; k <<= 1) {
        #pragma unroll 1
        for (int j = k >> 1; j > 0; j >>= 1) {
            #pragma unroll 1
            for (int q = lane_id(); q < P / 2; q += kWave) {
                const int i = ((q & ~(j - 1)) << 1) | (q & (j - 1));
                const int l = i | j;
                const Cand x = a[i], y = a[l];
                // best first where bit k of i is clear, worst first elsewhere
                const bool swap = (i & k) == 0 ? better(y.num, y.key, x.num, x.key) : better(x.num, x.key, y.num, y.key);
                if (swap) {
                    a[i] = y;
                    a[l] = x;
                }
            }
            wave_sync();
        }
    }
}

// Candidates wanted by a wave at once past which they go to the list as a
// batch (appended, then the list sorted and cut back to K) instead of one
// replacement and rescan each.  BATCH: the kernels whose waves see few
// combinations each (order 2, no pilot pass on small scans); in the others
// the extra code costs the scoring loops registers.
constexpr int kBatchOffer = 8;

template <bool BATCH = false>
EPI_DEV void tk_offer(TopK &t, Cand *list, bool valid, long long num, unsigned long long key, long long gthr) {
    bool want = valid && num >= gthr && (t.n < t.K || better(num, key, t.wn, t.wk));
    unsigned long long mask = __ballot(want);
    // counted once the list is full or a bound exists: the unbounded filling
    // of the lists at the start would only add contention
    if (mask && t.hist && !t.nohist && (t.n == t.K || gthr != (long long)0x8000000000000000ull))
        hist_add(t, want, num);
    const int cnt = __popcll(mask);
    if (BATCH && cnt >= kBatchOffer && tk_sort_size(t.n + cnt) <= t.cap) {
        wave_sync();
        if (want) list[t.n + (int)lane_prefix(mask)] = Cand{num, key};
        const int n2 = t.n + cnt;
        wave_sync();
        if (n2 < t.K) {
            t.n = n2;
            return;
        }
        tk_sort(list, n2);
        // the best K stay, the K-th best is the entry the next better
        // candidate replaces
        t.n = t.K;
        const Cand w = list[t.K - 1];
        t.wn = (long long)rfl64((unsigned long long)w.num);
        t.wk = rfl64(w.key);
        t.wi = t.K - 1;
        return;
    }
    while (mask) {
        const int src = __builtin_ctzll(mask);
        const long long cn = (long long)readlane64((unsigned long long)num, src);
        const unsigned long long ck = readlane64(key, src);
        if (t.n < t.K) {
            if (lane_id() == 0) list[t.n] = Cand{cn, ck};
            t.n++;
            if (t.n == t.K) {
                wave_sync();
                tk_recompute(t, list);
            }
        } else if (better(cn, ck, t.wn, t.wk)) {
            if (lane_id() == 0) list[t.wi] = Cand{cn, ck};
            wave_sync();
            tk_recompute(t, list);
        }
        mask &= mask - 1;
        if (t.n == t.K) mask &= __ballot(want && better(num, key, t.wn, t.wk));
    }
}

// Append the list's entries that can still be in the final best K to the
// task's candidate buffer, then empty the list.
EPI_DEV void tk_flush(TopK &t, const Cand *list, const Task &task) {
    wave_sync();
    const long long g = load_thr(task.thr);
    for (int base = 0; base < t.n; base += kWave) {
        const int i = base + lane_id();
        Cand c{0, 0};
        bool keep = false;
        if (i < t.n) {
            c = list[i];
            keep = c.num >= g;
        }
        unsigned long long m = __ballot(keep);
        unsigned cnt = (unsigned)__popcll(m);
        unsigned off = 0;
        if (lane_id() == 0 && cnt) off = atomicAdd(task.cand_count, cnt);
        off = __builtin_amdgcn_readfirstlane(off);
        unsigned pos = off + lane_prefix(m);
        if (keep && pos < task.cand_cap) task.cand[pos] = c;
    }
    wave_sync();
    t.n = 0;
}

typedef __attribute__((address_space(1))) const long long glong;

// One cell's contribution T(n0) + T(n1) - T(n0 + n1) for counts derived by
// inclusion-exclusion.  The table holds 2N + 1 entries and each class count
// is clamped to N, so no value can index past it.
EPI_DEV long long cell_term(const long long *T, int n0, int n1, unsigned N) {
    const unsigned a = min((unsigned)n0, N);
    const unsigned b = min((unsigned)n1, N);
    glong *g = (glong *)T;
    return g[a] + g[b] - g[a + b];
}

// Same for counts that are popcounts of one class each (n0 + n1 <= N).
EPI_DEV long long cell_term_counted(const long long *T, unsigned n0, unsigned n1) {
    glong *g = (glong *)T;
    return g[n0] + g[n1] - g[n0 + n1];
}

// ---------------------------------------------------------------------------
// Score screening.  A combination can only enter a wave's best-K list if its
// score reaches te (the task's global bound, or the list's current worst once
// the list is full).  The same cell terms summed from the 32-bit table t(n) =
// round(n ln n 2^tq) (the workgroup's LDS copy, reloaded when a chunk of work
// starts a dataset whose table fits) give the score to within one unit of
// 2^-tq per table value read, so combinations whose sum is below the bound
// by more than that skip the exact int64 sum; the exact path is unchanged.
// The sums are taken modulo 2^32: only the result, at most 2^30 in size,
// needs to fit.  Datasets whose table is not in LDS take the exact path for
// every combination.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) const unsigned lu32;
typedef __attribute__((address_space(3))) v4u lv4u;

// The table sits at LDS address 0 (checked when it is loaded), so an entry's
// address is its byte offset with no base to add.  LDS reads cannot fault;
// the counts of valid lanes are always in range.
EPI_DEV unsigned ltab(unsigned byte) { return *(lu32 *)(uintptr_t)byte; }

// The per-combination kernels take the exact table round(n ln n 2^shift),
// n = 0 .. N, at LDS address 0 when it fits: entry n is at byte 8n.
typedef __attribute__((address_space(3))) const long long lli64;
EPI_DEV long long cell_term_lds(unsigned n0, unsigned n1) {
    return *(lli64 *)(uintptr_t)(8u * n0) + *(lli64 *)(uintptr_t)(8u * n1) - *(lli64 *)(uintptr_t)(8u * (n0 + n1));
}

// Stage the genotype-0/1 rows of `nsnp` wave-uniform SNPs (snp_of(r) for row
// pair r) over words [w0, w0 + wn) of class c into the wave's LDS slot:
// slot[(2 * r + g) * cw + w].  One coalesced pass by all lanes; the counting
// loop then reads them with broadcast LDS loads instead of scalar loads.
template <class SnpOf>
EPI_DEV void stage_rows(lv4u *slot, gv4u *gm, long long Mp, int wbase, int w0, int wn, int cw, int nsnp,
                        SnpOf snp_of) {
    wave_sync();
    const int n = 2 * nsnp * wn;
    for (int e = lane_id(); e < n; e += kWave) {
        const int r2 = e / wn;
        const int w = e - r2 * wn;
        const int r = r2 >> 1, g = r2 & 1;
        slot[r2 * cw + w] = gm[((long long)(wbase + w0 + w) * 2 + g) * Mp + snp_of(r)];
    }
    wave_sync();
}

// Screening sum of CELLS cells of plain counts (entry n at byte 4n).
template <int CELLS>
EPI_DEV int screen_sum(const int (&F0)[CELLS], const int (&F1)[CELLS]) {
    unsigned p = 0, q = 0, qh = 0;
    #pragma unroll
    for (int x = 0; x < CELLS; ++x) {
        p = add3(p, ltab(4u * (unsigned)F0[x]), ltab(4u * (unsigned)F1[x]));
        // the subtracted terms in pairs
        if (x & 1) q = add3(q, qh, ltab(4u * (unsigned)(F0[x] + F1[x])));
        else qh = ltab(4u * (unsigned)(F0[x] + F1[x]));
    }
    return (int)(p - q - ((CELLS & 1) ? qh : 0u));
}

// Same for the signed cell form (matrix-core order 3, order 4 by reduced
// cells); with REV the table's mirrored half is in LDS and a B - 4n cell is
// its address there, else it is turned back into 4n.
template <int CELLS, bool REV>
EPI_DEV int screen_sum_signed(const unsigned (&F0)[CELLS], const unsigned (&F1)[CELLS], unsigned B) {
    const unsigned nB = 0u - B;
    unsigned p = 0, q = 0, qh = 0;
    #pragma unroll
    for (int x = 0; x < CELLS; ++x) {
        unsigned a0 = F0[x], a1 = F1[x], s;
        if (odd_twos(x)) {
            if constexpr (REV) {
                s = add3(a0, a1, nB);  // B - 4 (n0 + n1)
            } else {
                a0 = B - a0;
                a1 = B - a1;
                s = a0 + a1;
            }
        } else {
            s = a0 + a1;
        }
        p = add3(p, ltab(a0), ltab(a1));
        // the subtracted terms in pairs
        if (x & 1) q = add3(q, qh, ltab(s));
        else qh = ltab(s);
    }
    return (int)(p - q - qh);
}

// Same for the packed cell form of order 4 by reduced cells (both classes of
// a cell in one register, 4 n(cases) | 4 n(controls) << 16: each half is its
// entry's byte address).
template <int CELLS>
EPI_DEV int screen_sum_packed(const unsigned (&F)[CELLS]) {
    unsigned p = 0, q = 0, qh = 0;
    #pragma unroll
    for (int x = 0; x < CELLS; ++x) {
        const unsigned a0 = F[x] & 0xffffu, a1 = F[x] >> 16;
        p = add3(p, ltab(a0), ltab(a1));
        // the subtracted terms in pairs
        if (x & 1) q = add3(q, qh, ltab(a0 + a1));
        else qh = ltab(a0 + a1);
    }
    return (int)(p - q - ((CELLS & 1) ? qh : 0u));
}

// Smallest screening sum of a combination whose num can reach te, for sums
// of `reads` table values.  Each table value and each exact term is within
// 1/2 of its scaled n ln n, so a sum and the num it screens for differ by at
// most reads units of 2^-tq (tq <= shift); one more unit covers the rounding
// of the scaled bound.
EPI_DEV int screen_bound(long long te, long long score_const, int shift, int tq, int reads) {
    if (te == (long long)0x8000000000000000ull) return (int)0x80000000u;
    const double v = ldexp((double)(te - score_const), tq - shift);
    return (int)floor(v) - reads - 1;
}

EPI_DEV long long entry_bound(const TopK &tk, long long gthr) {
    return tk.n < tk.K ? gthr : (tk.wn > gthr ? tk.wn : gthr);
}

// Pilot pass over an item: the wave's best screening sum S (best over its
// lanes' combinations; INT_MIN: none) becomes one histogram count.  S is
// within `reads` units (2^-tq) of (num - score_const) 2^(tq - shift) (each
// table value within one unit of its n ln n, as in screen_bound), so
// score_const + (S - reads - 1) 2^(shift - tq) is below that combination's
// num; one atomic per wave, and the K-th best of such maxima is close to the
// K-th best of all the item's combinations.
EPI_DEV void pilot_count(TopK &tk, const Task &t, int best, int reads) {
    #pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(best, off);
        best = o > best ? o : best;
    }
    hist_add(tk, lane_id() == 0 && best != (int)0x80000000u,
             t.score_const + (long long)(best - reads - 1) * (1ll << (t.ds.shift - t.ds.tq)));
}

// ---------------------------------------------------------------------------
// kF2 / kF2Emit / kF2Fold: order 2.  A work item is (block of NP SNPs i,
// block of 64 SNPs m > i); lane = m.  Reduced cells (a, d) in {0,1}^2 per
// class, scored (kF2), written to the pair sub-table (kF2Emit), or both
// (kF2Fold: a scan of all orders takes its order-2 results from the pair
// sub-table pass of its higher orders instead of counting the pairs twice).
// ---------------------------------------------------------------------------
template <int NP, bool EMIT, bool LDS, bool SCORE = !EMIT, bool CHECK = false, bool PILOT = false>
EPI_DEV void item_f2(const Task &t, unsigned long long local, TopK &tk, Cand *list, long long gthr, v4u *stage,
                     int stage_cap) {
    static_assert(!PILOT || (LDS && SCORE && !EMIT && !CHECK), "the pilot pass scores from the LDS table");
    const DsView d = t.ds;
    int pilot_best = (int)0x80000000u;  // PILOT: the lane's best screening sum
    const unsigned long long dsc = t.items[local];
    const int ib = uni((int)((dsc >> 20) & 0xfffffu));
    const int mb = uni((int)(dsc & 0xfffffu));
    const int i0 = ib * NP;
    const int lane = lane_id();
    const int m = i0 + 1 + mb * kWave + lane;
    const bool mv = m < d.M;
    const int m_ld = mv ? m : d.Mp - 1;
    int ip[NP];
    #pragma unroll
    for (int p = 0; p < NP; ++p) ip[p] = uni(min(i0 + p, d.M - 1));

    gv4u *gm = (gv4u *)d.masks;
    unsigned acc[NP][2][4];
    #pragma unroll
    for (int p = 0; p < NP; ++p)
        #pragma unroll
        for (int c = 0; c < 2; ++c)
            #pragma unroll
            for (int e = 0; e < 4; ++e) acc[p][c][e] = 0;

    const long long Mp = d.Mp;
    lv4u *slot = (lv4u *)stage;
    const int cw = stage_cap / (2 * NP);  // words (x4) per staged chunk
    #pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int W = d.w4[c];
        long long off = (long long)d.wbase[c] * 2 * Mp;
        v4u m0n = gm[off + m_ld];
        v4u m1n = gm[off + Mp + m_ld];
        for (int w0 = 0; w0 < W; w0 += cw) {
            const int wn = min(cw, W - w0);
            stage_rows(slot, gm, Mp, d.wbase[c], w0, wn, cw, NP, [&](int r) { return min(i0 + r, d.M - 1); });
        for (int w = 0; w < wn; ++w, off += 2 * Mp) {
            const v4u m0 = m0n;
            const v4u m1 = m1n;
            // next iteration's lane rows (the last iteration re-reads its own)
            const long long offn = w0 + w + 1 < W ? off + 2 * Mp : off;
            m0n = gm[offn + m_ld];
            m1n = gm[offn + Mp + m_ld];
            #pragma unroll
            for (int p = 0; p < NP; ++p) {
                const v4u a0 = slot[(2 * p + 0) * cw + w];
                const v4u a1 = slot[(2 * p + 1) * cw + w];
                #pragma unroll
                for (int q = 0; q < 4; ++q) {
                    acc[p][c][0] = bcnt_acc(a0[q] & m0[q], acc[p][c][0]);
                    acc[p][c][1] = bcnt_acc(a0[q] & m1[q], acc[p][c][1]);
                    acc[p][c][2] = bcnt_acc(a1[q] & m0[q], acc[p][c][2]);
                    acc[p][c][3] = bcnt_acc(a1[q] & m1[q], acc[p][c][3]);
                }
            }
        }
        }
    }

    const v4u *single4 = (const v4u *)d.single;
    const v4u sm = single4[m_ld];
    #pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int i = i0 + p;
        const bool valid = mv && i < m && i <= d.M - 2;
        if constexpr (EMIT) {
            if (valid) {
                v4u *pv = (v4u *)t.pairs;
                const unsigned long long r = t.pair_colex ? colex2(i, m) : lexpair(i, m, d.M);
                if (t.pair_colex) {
                    // order 4 by reduced cells: one word per cell, both classes
                    // (4 n(cases) | 4 n(controls) << 16)
                    pv[r] = v4u{(acc[p][0][0] << 2) | (acc[p][1][0] << 18), (acc[p][0][1] << 2) | (acc[p][1][1] << 18),
                                (acc[p][0][2] << 2) | (acc[p][1][2] << 18), (acc[p][0][3] << 2) | (acc[p][1][3] << 18)};
                } else {
                const int sh = t.cell_shift;
                v4u c0 = v4u{acc[p][0][0] << sh, acc[p][0][1] << sh, acc[p][0][2] << sh, acc[p][0][3] << sh};
                v4u c1 = v4u{acc[p][1][0] << sh, acc[p][1][1] << sh, acc[p][1][2] << sh, acc[p][1][3] << sh};
                if (t.cell_neg) {
                    c0 = t.cell_bias - c0;
                    c1 = t.cell_bias - c1;
                } else {
                    c0 += t.cell_bias;
                    c1 += t.cell_bias;
                }
                pv[2 * r + 0] = c0;
                pv[2 * r + 1] = c1;
                }
            }
        }
        if constexpr (SCORE) {
            const v4u si = single4[ip[p]];
            int F[2][9];
            #pragma unroll
            for (int c = 0; c < 2; ++c) {
                F[c][0] = acc[p][c][0];
                F[c][1] = acc[p][c][1];
                F[c][3] = acc[p][c][2];
                F[c][4] = acc[p][c][3];
                F[c][2] = si[2 * c + 0];
                F[c][5] = si[2 * c + 1];
                F[c][6] = sm[2 * c + 0];
                F[c][7] = sm[2 * c + 1];
                F[c][8] = d.ncls[c];
                mobius2(F[c]);
            }
            if constexpr (PILOT) {
                if (valid) {
                    const int S = screen_sum<9>(F[0], F[1]);
                    pilot_best = S > pilot_best ? S : pilot_best;
                }
                continue;
            }
            if constexpr (CHECK) {
                const int cc[2] = {i, m};
                digest_add(tk, valid, combo_hash<2>(cc), table_sum<9>(F[0], F[1]));
            }
            bool pass = valid;
            if constexpr (LDS) {
                const int sb = screen_bound(entry_bound(tk, gthr), t.score_const, d.shift, d.tq, 27);
                pass = pass && screen_sum<9>(F[0], F[1]) >= sb;
            }
            if (__ballot(pass)) {
                long long num = t.score_const;
                #pragma unroll
                for (int x = 0; x < 9; ++x) num += cell_term(d.tlog, F[0][x], F[1][x], (unsigned)d.N);
                const unsigned long long key = ((unsigned long long)i << 32) | (unsigned long long)m;
                tk_offer<true>(tk, list, pass, num, key, gthr);
            }
        }
    }
    if constexpr (PILOT) pilot_count(tk, t, pilot_best, 27);
}

// ---------------------------------------------------------------------------
// kF3: order 3.  A work item is (j, block of NP SNPs i < j, block of 64 SNPs
// m > j); lane = m.  Reduced cells (a, b, d) in {0,1}^3 per class; every
// other cell comes from the pair sub-table and the single-SNP counts.
// ---------------------------------------------------------------------------
template <int NP, bool LDS, bool CHECK = false>
EPI_DEV void item_f3(const Task &t, unsigned long long local, TopK &tk, Cand *list, long long gthr, v4u *stage,
                     int stage_cap) {
    const DsView d = t.ds;
    const unsigned long long dsc = t.items[local];
    const int j = uni((int)((dsc >> 40) & 0xfffffu));
    const int ib = uni((int)((dsc >> 20) & 0xfffffu));
    const int mb = uni((int)(dsc & 0xfffffu));
    const int i0 = ib * NP;
    const int lane = lane_id();
    const int m = j + 1 + mb * kWave + lane;
    const bool mv = m < d.M;
    const int m_ld = mv ? m : d.Mp - 1;
    int ip[NP];
    #pragma unroll
    for (int p = 0; p < NP; ++p) ip[p] = uni(min(i0 + p, j - 1));

    // sub-table rows the epilogue needs, issued before the counting loop
    const v4u *single4 = (const v4u *)d.single;
    const v4u *pair4 = (const v4u *)t.pairs;
    const v4u sm = single4[m_ld];
    const unsigned long long rjm = mv ? lexpair(j, m, d.M) : 0ull;
    const v4u pjm0 = pair4[2 * rjm], pjm1 = pair4[2 * rjm + 1];
    unsigned long long rim = (mv && i0 < j) ? lexpair(i0, m, d.M) : 0ull;
    v4u pim_n0 = pair4[2 * rim], pim_n1 = pair4[2 * rim + 1];

    gv4u *gm = (gv4u *)d.masks;
    unsigned acc[NP][2][8];
    #pragma unroll
    for (int p = 0; p < NP; ++p)
        #pragma unroll
        for (int c = 0; c < 2; ++c)
            #pragma unroll
            for (int e = 0; e < 8; ++e) acc[p][c][e] = 0;

    const long long Mp = d.Mp;
    lv4u *slot = (lv4u *)stage;
    const int cw = stage_cap / (2 * (NP + 1));  // words (x4) per staged chunk
    #pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int W = d.w4[c];
        long long off = (long long)d.wbase[c] * 2 * Mp;
        v4u m0n = gm[off + m_ld];
        v4u m1n = gm[off + Mp + m_ld];
        for (int w0 = 0; w0 < W; w0 += cw) {
            const int wn = min(cw, W - w0);
            // row pair 0 = j, row pair 1 + p = i0 + p
            stage_rows(slot, gm, Mp, d.wbase[c], w0, wn, cw, NP + 1,
                       [&](int r) { return r == 0 ? j : min(i0 + r - 1, j - 1); });
        for (int w = 0; w < wn; ++w, off += 2 * Mp) {
            const v4u m0 = m0n;
            const v4u m1 = m1n;
            // next iteration's lane rows (the last iteration re-reads its own)
            const long long offn = w0 + w + 1 < W ? off + 2 * Mp : off;
            m0n = gm[offn + m_ld];
            m1n = gm[offn + Mp + m_ld];
            const v4u b0 = slot[0 * cw + w];
            const v4u b1 = slot[1 * cw + w];
            #pragma unroll
            for (int p = 0; p < NP; ++p) {
                const v4u a0 = slot[(2 * p + 2) * cw + w];
                const v4u a1 = slot[(2 * p + 3) * cw + w];
                #pragma unroll
                for (int q = 0; q < 4; ++q) {
                    acc[p][c][0] = bcnt_acc(a0[q] & b0[q] & m0[q], acc[p][c][0]);
                    acc[p][c][1] = bcnt_acc(a0[q] & b0[q] & m1[q], acc[p][c][1]);
                    acc[p][c][2] = bcnt_acc(a0[q] & b1[q] & m0[q], acc[p][c][2]);
                    acc[p][c][3] = bcnt_acc(a0[q] & b1[q] & m1[q], acc[p][c][3]);
                    acc[p][c][4] = bcnt_acc(a1[q] & b0[q] & m0[q], acc[p][c][4]);
                    acc[p][c][5] = bcnt_acc(a1[q] & b0[q] & m1[q], acc[p][c][5]);
                    acc[p][c][6] = bcnt_acc(a1[q] & b1[q] & m0[q], acc[p][c][6]);
                    acc[p][c][7] = bcnt_acc(a1[q] & b1[q] & m1[q], acc[p][c][7]);
                }
            }
        }
        }
    }

    const v4u sj = single4[j];
    #pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int i = i0 + p;
        const bool valid = mv && i < j;
        const v4u pim0 = pim_n0, pim1 = pim_n1;
        if (p + 1 < NP) {
            // next prefix's pair row, in flight while this one is scored
            rim = (mv && i + 1 < j) ? lexpair(i + 1, m, d.M) : 0ull;
            pim_n0 = pair4[2 * rim];
            pim_n1 = pair4[2 * rim + 1];
        }
        const v4u si = single4[ip[p]];
        const unsigned long long rij = lexpair(ip[p], j, d.M);
        int F[2][27];
        #pragma unroll
        for (int c = 0; c < 2; ++c) {
            const v4u pij = pair4[2 * rij + c];
            const v4u pim = c == 0 ? pim0 : pim1;
            const v4u pjm = c == 0 ? pjm0 : pjm1;
            // F[a*9 + b*3 + e]; index 2 on an axis = marginal over that SNP
            #pragma unroll
            for (int a = 0; a < 2; ++a)
                #pragma unroll
                for (int b = 0; b < 2; ++b)
                    #pragma unroll
                    for (int e = 0; e < 2; ++e) F[c][9 * a + 3 * b + e] = acc[p][c][4 * a + 2 * b + e];
            #pragma unroll
            for (int a = 0; a < 2; ++a)
                #pragma unroll
                for (int b = 0; b < 2; ++b) F[c][9 * a + 3 * b + 2] = pij[2 * a + b];
            #pragma unroll
            for (int a = 0; a < 2; ++a)
                #pragma unroll
                for (int e = 0; e < 2; ++e) F[c][9 * a + 6 + e] = pim[2 * a + e];
            #pragma unroll
            for (int b = 0; b < 2; ++b)
                #pragma unroll
                for (int e = 0; e < 2; ++e) F[c][18 + 3 * b + e] = pjm[2 * b + e];
            F[c][9 * 0 + 8] = si[2 * c + 0];
            F[c][9 * 1 + 8] = si[2 * c + 1];
            F[c][18 + 2] = sj[2 * c + 0];
            F[c][18 + 5] = sj[2 * c + 1];
            F[c][24] = sm[2 * c + 0];
            F[c][25] = sm[2 * c + 1];
            F[c][26] = d.ncls[c];
            mobius3(F[c]);
        }
        if constexpr (CHECK) {
            const int cc[3] = {i, j, m};
            digest_add(tk, valid, combo_hash<3>(cc), table_sum<27>(F[0], F[1]));
        }
        bool pass = valid;
        if constexpr (LDS) {
            const int sb = screen_bound(entry_bound(tk, gthr), t.score_const, d.shift, d.tq, 81);
            pass = pass && screen_sum<27>(F[0], F[1]) >= sb;
        }
        if (__ballot(pass)) {
            long long num = t.score_const;
            #pragma unroll
            for (int x = 0; x < 27; ++x) num += cell_term(d.tlog, F[0][x], F[1][x], (unsigned)d.N);
            const unsigned long long key =
                ((unsigned long long)i << 42) | ((unsigned long long)j << 21) | (unsigned long long)m;
            tk_offer(tk, list, pass, num, key, gthr);
        }
    }
}

// ---------------------------------------------------------------------------
// kF3 with np = kNpMfma: order 3 counted by matrix cores.  A work item is
// (j, block of 16 SNPs i, block of 32 SNPs m); every (i, j, m) with i < j < m
// in it is one triplet.  Counts of individuals with genotypes (a, b, d) at
// (i, j, m) are dot products of 0/1 indicator rows, so the reduced cells of a
// class are the products (X_i . x_{j,b})^T X_m over its individuals, one
// matrix-core product per step of individuals, b and d: rows (i, a) are A,
// the rows of genotype b of SNP j mask A, rows (m, d) are B.  With 4-bit
// float operands (1.0 = 0x2; v_mfma_scale_f32_32x32x64_f8f6f4, 64
// individuals per step) products are 0 or 4 and sums stay below 2^24, so the
// float accumulators hold the exact counts; 8-bit integer operands
// (v_mfma_i32_32x32x32_i8, 32 per step) give the same integers.  B holds 4
// for a set bit, so the sums are 4 n: a count is then the byte offset of its
// entry in the float screening table.  In the 32 x 32 result,
// lane l holds column l % 32 (SNP m) and rows 8 (r / 4) + 4 (l / 32) + r % 4
// of its 16 registers r, i.e. both genotypes a of eight SNPs i; the epilogue
// is that of the popcount kernel.
// ---------------------------------------------------------------------------
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Descriptor word 3 of a raw (untyped, unswizzled) gfx9 buffer.
constexpr int kBufWord3 = 0x00020000;
// Steps of 64 individuals in flight per operand stream.
constexpr int kQDepth = kQStepMultiple;
// Steps whose j-mask rows are staged in LDS at a time (4 entries per step).
constexpr int kQSeg = kQStageSteps;

EPI_DEV v4u qload(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(v4u, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

typedef int v16i __attribute__((ext_vector_type(16)));

// Operand format of the matrix-core order-3 kernel.
//   I8 = false: 4-bit floats, 64 individuals per step, float32 sums;
//   I8 = true:  8-bit integers, 32 individuals per step, int32 sums.
template <bool I8>
struct QFmt;

template <>
struct QFmt<false> {
    typedef v16f acc_t;
    static EPI_DEV const v4u *qa(const DsView &d) { return d.qa; }
    static EPI_DEV const v4u *qb(const DsView &d) { return d.qb; }
    static EPI_DEV int ks(const DsView &d, int c) { return d.ks[c]; }
    // sb: exponent scale of the B operand (E8M0, 127 = 2^0)
    static EPI_DEV acc_t mma(v4u a, v4u b, acc_t c, int sb = 127) {
        const v8i a8 = {(int)a[0], (int)a[1], (int)a[2], (int)a[3], 0, 0, 0, 0};
        const v8i b8 = {(int)b[0], (int)b[1], (int)b[2], (int)b[3], 0, 0, 0, 0};
        // formats 4 / 4: e2m1 for both operands; A scale 127 = 2^0
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, c, 4, 4, 0, 127, 0, sb);
    }
};

template <>
struct QFmt<true> {
    typedef v16i acc_t;
    static EPI_DEV const v4u *qa(const DsView &d) { return d.qa8; }
    static EPI_DEV const v4u *qb(const DsView &d) { return d.qb8; }
    static EPI_DEV int ks(const DsView &d, int c) { return d.ks8[c]; }
    static EPI_DEV acc_t mma(v4u a, v4u b, acc_t c, int = 127) {
        return __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(v4i, a), __builtin_bit_cast(v4i, b), c, 0, 0,
                                                     0);
    }
};

// ---------------------------------------------------------------------------
// kF2 with prefix block kNpMfma: order 2 on the matrix cores, the products of
// the order-3 kernel below without the middle SNP's mask.  A work item is
// (block ib of 32 SNPs i, block mb of 32 SNPs m); per step and class four
// products, A0 and A1 (32 rows each: the genotype-0 and -1 rows of the
// item's two 16-SNP blocks of i) times B0 and B1 (the 32 m's genotype-0 and
// -1 rows), 4 n per cell: four operand loads feed four products (two A
// blocks, so that the loads per product are those of the order-3 kernel).
// Lane l holds column m = 32 mb + l % 32 and both genotypes a of eight SNPs
// i of each A block (the layout of item_f3m); the epilogue is item_f2's.
// ---------------------------------------------------------------------------
template <bool LDS, bool CHECK = false, bool PILOT = false>
EPI_DEV void item_f2m(const Task &t, unsigned long long local, TopK &tk, Cand *list, long long gthr) {
    static_assert(!PILOT || (LDS && !CHECK), "the pilot pass scores from the LDS table");
    typedef QFmt<false> Q;
    int pilot_best = (int)0x80000000u;  // PILOT: the lane's best screening sum
    const DsView d = t.ds;
    const unsigned long long dsc = t.items[local];
    const int ib = uni((int)((dsc >> 20) & 0xfffffu));
    const int mb = uni((int)(dsc & 0xfffffu));
    const int lane = lane_id(), h = lane >> 5;
    const int m = mb * 32 + (lane & 31);
    const bool mv = m < d.M;
    const int m_ld = mv ? m : d.M - 1;
    const int KS = Q::ks(d, 0) + Q::ks(d, 1);
    const int blk = KS * 1024;  // bytes of one row block
    const v4u *qa = Q::qa(d), *qb = Q::qb(d);
    // the second 16-SNP block of i; past the operand copy's last block (its
    // SNPs would be M or more) the first block again, its lanes invalid
    const int nib = (d.M + 15) / 16;
    const int ib1 = 2 * ib + 1 < nib ? 2 * ib + 1 : 2 * ib;
    __amdgpu_buffer_rsrc_t rA[2];
    rA[0] = __builtin_amdgcn_make_buffer_rsrc((void *)(qa + (long long)(2 * ib) * KS * 64), 0, blk, kBufWord3);
    rA[1] = __builtin_amdgcn_make_buffer_rsrc((void *)(qa + (long long)ib1 * KS * 64), 0, blk, kBufWord3);
    const __amdgpu_buffer_rsrc_t rB0 =
        __builtin_amdgcn_make_buffer_rsrc((void *)(qb + (long long)(2 * mb) * KS * 64), 0, blk, kBufWord3);
    const __amdgpu_buffer_rsrc_t rB1 =
        __builtin_amdgcn_make_buffer_rsrc((void *)(qb + (long long)(2 * mb + 1) * KS * 64), 0, blk, kBufWord3);
    const int vo = lane * 16;
    typename Q::acc_t acc[2][2][2];  // [class][A block][genotype of m]
    #pragma unroll
    for (int c = 0; c < 2; ++c)
        #pragma unroll
        for (int a = 0; a < 2; ++a)
            #pragma unroll
            for (int e = 0; e < 2; ++e) acc[c][a][e] = (typename Q::acc_t){};
    // the software pipeline of item_f3m: kQDepth steps in flight, both
    // classes one stream
    const int ks0 = Q::ks(d, 0);
    v4u bA0[kQDepth], bA1[kQDepth], bB0[kQDepth], bB1[kQDepth];
    #pragma unroll
    for (int u = 0; u < kQDepth; ++u) {
        const int so = min(u, KS - 1) * 1024;
        bA0[u] = qload(rA[0], vo, so);
        bA1[u] = qload(rA[1], vo, so);
        bB0[u] = qload(rB0, vo, so);
        bB1[u] = qload(rB1, vo, so);
        __builtin_amdgcn_sched_barrier(0);
    }
    #pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int c0 = c == 0 ? 0 : ks0;
        const int cn = Q::ks(d, c);
        #pragma unroll 1
        for (int k = 0; k < cn; k += kQDepth) {
            const int g = c0 + k;
            #pragma unroll
            for (int u = 0; u < kQDepth; ++u) {
                acc[c][0][0] = Q::mma(bA0[u], bB0[u], acc[c][0][0]);
                acc[c][0][1] = Q::mma(bA0[u], bB1[u], acc[c][0][1]);
                acc[c][1][0] = Q::mma(bA1[u], bB0[u], acc[c][1][0]);
                acc[c][1][1] = Q::mma(bA1[u], bB1[u], acc[c][1][1]);
                const int so = min(g + u + kQDepth, KS - 1) * 1024;
                bA0[u] = qload(rA[0], vo, so);
                bA1[u] = qload(rA[1], vo, so);
                bB0[u] = qload(rB0, vo, so);
                bB1[u] = qload(rB1, vo, so);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    const v4u *single4 = (const v4u *)d.single;
    const v4u sm = single4[m_ld];
    // the eight pairs of a lane in each A block (a function per block, so
    // that each loop over them unrolls and every accumulator index is a
    // constant)
    auto score_block = [&](const typename Q::acc_t (&c0)[2], const typename Q::acc_t (&c1)[2], int ab)
                           __attribute__((always_inline)) {
        const int i_base = ib * 32 + 16 * ab + 2 * h;
        #pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i_base + 4 * (u >> 1) + (u & 1);
            const int r0 = 4 * (u >> 1) + 2 * (u & 1);
            const bool valid = mv && i < m;
            const v4u si = single4[min(i, d.M - 1)];
            int F[2][9];
            #pragma unroll
            for (int c = 0; c < 2; ++c) {
                #pragma unroll
                for (int a = 0; a < 2; ++a)
                    #pragma unroll
                    for (int e = 0; e < 2; ++e) F[c][3 * a + e] = (int)(c == 0 ? c0 : c1)[e][r0 + a] >> kQScaleShift;
                F[c][2] = si[2 * c + 0];
                F[c][5] = si[2 * c + 1];
                F[c][6] = sm[2 * c + 0];
                F[c][7] = sm[2 * c + 1];
                F[c][8] = d.ncls[c];
                mobius2(F[c]);
            }
            if constexpr (PILOT) {
                if (valid) {
                    const int S = screen_sum<9>(F[0], F[1]);
                    pilot_best = S > pilot_best ? S : pilot_best;
                }
                continue;
            }
            if constexpr (CHECK) {
                const int cc[2] = {i, m};
                digest_add(tk, valid, combo_hash<2>(cc), table_sum<9>(F[0], F[1]));
            }
            bool pass = valid;
            if constexpr (LDS) {
                const int sb = screen_bound(entry_bound(tk, gthr), t.score_const, d.shift, d.tq, 27);
                pass = pass && screen_sum<9>(F[0], F[1]) >= sb;
            }
            if (__ballot(pass)) {
                long long num = t.score_const;
                #pragma unroll
                for (int x = 0; x < 9; ++x) num += cell_term(d.tlog, F[0][x], F[1][x], (unsigned)d.N);
                const unsigned long long key = ((unsigned long long)i << 32) | (unsigned long long)m;
                tk_offer<true>(tk, list, pass, num, key, gthr);
            }
        }
    };
    score_block(acc[0][0], acc[1][0], 0);
    score_block(acc[0][1], acc[1][1], 1);
    if constexpr (PILOT) pilot_count(tk, t, pilot_best, 27);
}

// PILOT: the histogram-only pass over an item (needs the screening table in
// LDS): lower bounds of the scores are counted, nothing is offered.
template <bool LDS, bool REV, bool I8, bool EMIT = false, bool CHECK = false, int NJ = 1, bool PILOT = false>
EPI_DEV void item_f3m(const Task &t, unsigned long long local, TopK &tk, Cand *list, long long gthr, v4u *stage) {
    static_assert(NJ == 1 || (NJ == 2 && !EMIT && !I8), "two middle SNPs per item: 4-bit scoring kernel only");
    typedef QFmt<I8> Q;
    // PK (two middle SNPs): one accumulator per tile for both classes, the
    // control steps' products scaled by 2^(T - 2), so the tile holds
    // 4 n(cases) + 2^T n(controls) (q3_pack_shift; the host takes this kernel
    // only where q3_pack_fits)
    constexpr bool PK = NJ == 2;
    constexpr int NC = PK ? 1 : 2;
    const int T = PK ? q3_pack_shift(t.ds.ncls[0]) : 0;
    const DsView d = t.ds;
    const unsigned long long dsc = t.items[local];
    const int j = uni((int)((dsc >> 40) & 0xfffffu));
    const int ib = uni((int)((dsc >> 20) & 0xfffffu));
    const int mb = uni((int)(dsc & 0xfffffu));
    const int lane = lane_id(), h = lane >> 5;
    const int m = mb * 32 + (lane & 31);
    // The item's middle SNPs jv[0] = j and (NJ = 2) jv[1] = j + 1, which
    // share the i and m blocks and so every operand load of the counting
    // loop.  jc is a middle SNP below M - 1 for the sub-table reads of lanes
    // that have no valid triplet (jv[1] may be M - 1).
    int jv[NJ], jc[NJ], m_ld[NJ];
    bool mv[NJ];
    #pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        jv[jj] = j + jj;
        jc[jj] = min(jv[jj], d.M - 2);
        mv[jj] = m > jv[jj] && m < d.M;
        m_ld[jj] = mv[jj] ? m : jc[jj] + 1;
    }

    // sub-table rows the epilogue needs, issued before the counting loop; all
    // counts below are 4 n, in the signed form of the epilogue (the pair
    // sub-table is written that way, singles and class sizes are put in it
    // here)
    gv4u *single4 = (gv4u *)d.single;
    gv4u *pair4 = (gv4u *)t.pairs;
    const unsigned B = q3_bias(d.N), B4 = 4u * B;
    const v4u sm = (single4[m_ld[0]] << kQScaleShift) - B4;
    const unsigned nall[2] = {13u * B - ((unsigned)d.ncls[0] << kQScaleShift),
                              13u * B - ((unsigned)d.ncls[1] << kQScaleShift)};
    v4u sj[NJ], pjm0[NJ], pjm1[NJ];
    #pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        sj[jj] = (((cv4u *)d.single)[jv[jj]] << kQScaleShift) - B4;  // uniform: a scalar load
        const unsigned long long rjm = pair_row(jc[jj], d.M) + (unsigned)(m_ld[jj] - jc[jj] - 1);
        pjm0[jj] = pair4[2 * rjm];
        pjm1[jj] = pair4[2 * rjm + 1];
    }

    // operands through buffer descriptors (scalar registers): a lane adds
    // its own constant byte offset and a step adds a scalar one, so a step
    // costs no vector address arithmetic
    const int KS = Q::ks(d, 0) + Q::ks(d, 1);
    const int blk = KS * 1024;  // bytes of one row block
    const v4u *qa = Q::qa(d), *qb = Q::qb(d);
    const __amdgpu_buffer_rsrc_t rA =
        __builtin_amdgcn_make_buffer_rsrc((void *)(qa + (long long)ib * KS * 64), 0, blk, kBufWord3);
    __amdgpu_buffer_rsrc_t rJ[NJ];
    #pragma unroll
    for (int jj = 0; jj < NJ; ++jj)
        rJ[jj] = __builtin_amdgcn_make_buffer_rsrc((void *)(qa + (long long)(jv[jj] >> 4) * KS * 64), 0, blk,
                                                   kBufWord3);
    const __amdgpu_buffer_rsrc_t rB0 =
        __builtin_amdgcn_make_buffer_rsrc((void *)(qb + (long long)(2 * mb) * KS * 64), 0, blk, kBufWord3);
    const __amdgpu_buffer_rsrc_t rB1 =
        __builtin_amdgcn_make_buffer_rsrc((void *)(qb + (long long)(2 * mb + 1) * KS * 64), 0, blk, kBufWord3);
    const int vo = lane * 16;
    typename Q::acc_t acc[NJ][NC][2][2];
    #pragma unroll
    for (int jj = 0; jj < NJ; ++jj)
        #pragma unroll
        for (int c = 0; c < NC; ++c)
            #pragma unroll
            for (int b = 0; b < 2; ++b)
                #pragma unroll
                for (int e = 0; e < 2; ++e) acc[jj][c][b][e] = (typename Q::acc_t){};
    // Software pipeline: the operands of kQDepth steps are in flight while a
    // step is multiplied (a step's products take far less time than a load
    // from L2).  The steps of both classes form one stream, class 0's first
    // as in the operand copies (each class has a multiple of kQDepth steps,
    // zero-padded), so the pipeline runs on across the class boundary and an
    // item waits for operands only at its start.  Scheduling barriers keep
    // the loads in step order, each step's refills right after its products:
    // left alone, the scheduler sinks all refills to the end of the unrolled
    // block, and the loop then waits for every load in flight at its top.
    // The two mask rows of a middle SNP are the same for every lane of a half
    // wave: they are staged once per segment of kQSeg steps in the wave's LDS
    // slot (entry jj 4 kQSeg + 4 step + 2 h + b) and read back with broadcast
    // loads.
    lv4u *slot = (lv4u *)stage;
    const int ks0 = Q::ks(d, 0);
    v4u bA[kQDepth], bB0[kQDepth], bB1[kQDepth];
    #pragma unroll
    for (int u = 0; u < kQDepth; ++u) {
        const int so = min(u, KS - 1) * 1024;
        bA[u] = qload(rA, vo, so);
        bB0[u] = qload(rB0, vo, so);
        bB1[u] = qload(rB1, vo, so);
        __builtin_amdgcn_sched_barrier(0);
    }
    // mask rows of the segment [base, base + kQSeg) of the stream
    auto stage_masks = [&](int base) __attribute__((always_inline)) {
        const int n = min(kQSeg, KS - base);
        wave_sync();  // the slot's previous rows have been read
        // all loads issued at once, no branch between them (entries past the
        // segment repeat its last step's; the slot has room for them)
        #pragma unroll
        for (int jj = 0; jj < NJ; ++jj)
            #pragma unroll
            for (int e0 = 0; e0 < 4 * kQSeg; e0 += kWave) {
                const int e = min(e0 + lane, 4 * n - 1);
                const int vje = (((e >> 2) * 64) + 32 * ((e >> 1) & 1) + 2 * (jv[jj] & 15) + (e & 1)) * 16;
                slot[jj * 4 * kQSeg + e0 + lane] = qload(rJ[jj], vje, base * 1024);
            }
        wave_sync();
    };
    int seg = 0;
    stage_masks(0);
    #pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int c0 = c == 0 ? 0 : ks0;
        const int cn = Q::ks(d, c);
        const int cc = PK ? 0 : c;                      // accumulator set of the class
        const int bsc = PK && c == 1 ? 125 + T : 127;   // B scale: 2^(T - 2) for PK's controls
        #pragma unroll 1
        for (int k = 0; k < cn; k += kQDepth) {
            const int g = c0 + k;  // the group's first step in the stream
            if (g >= seg + kQSeg) {
                seg += kQSeg;
                stage_masks(seg);
            }
            #pragma unroll
            for (int u = 0; u < kQDepth; ++u) {
                #pragma unroll
                for (int jj = 0; jj < NJ; ++jj) {
                    const int js = jj * 4 * kQSeg + 4 * (g - seg + u) + 2 * h;
                    const v4u J0 = slot[js], J1 = slot[js + 1];
                    const v4u A0 = bA[u] & J0, A1 = bA[u] & J1;
                    acc[jj][cc][0][0] = Q::mma(A0, bB0[u], acc[jj][cc][0][0], bsc);
                    acc[jj][cc][0][1] = Q::mma(A0, bB1[u], acc[jj][cc][0][1], bsc);
                    acc[jj][cc][1][0] = Q::mma(A1, bB0[u], acc[jj][cc][1][0], bsc);
                    acc[jj][cc][1][1] = Q::mma(A1, bB1[u], acc[jj][cc][1][1], bsc);
                }
                // refill with the step kQDepth ahead in the stream (the last
                // steps re-read the stream's last step)
                const int so = min(g + u + kQDepth, KS - 1) * 1024;
                bA[u] = qload(rA, vo, so);
                bB0[u] = qload(rB0, vo, so);
                bB1[u] = qload(rB1, vo, so);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    wave_sync();  // the slot's rows have been read

    if constexpr (EMIT) {
        // triplet sub-table: the 8 cells 4a + 2b + d of the lane's eight
        // triplets at their colex ranks, both classes of a cell in one word
        // (the sums are 4n: 4 n(cases) | 4 n(controls) << 16, the packed form
        // of order 4 by reduced cells)
        gv4u *tv = (gv4u *)t.triples;
        #pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = ib * 16 + 2 * h + 4 * (u >> 1) + (u & 1);
            const int r0 = 4 * (u >> 1) + 2 * (u & 1);
            if (mv[0] && i < j) {
                v4u *dst = (v4u *)(tv + 2 * colex3(i, j, m));
                #pragma unroll
                for (int a = 0; a < 2; ++a) {
                    auto pk = [&](int b, int e) {
                        return (unsigned)(int)acc[0][0][b][e][r0 + a] | ((unsigned)(int)acc[0][NC - 1][b][e][r0 + a] << 16);
                    };
                    dst[a] = v4u{pk(0, 0), pk(0, 1), pk(1, 0), pk(1, 1)};
                }
            }
        }
        return;
    }

    // Cells F[c][9a + 3b + e] (digit 2: marginal over that SNP, genotype 2
    // once the inclusion-exclusion has run) in the signed form: a cell with
    // an odd number of digits 2 is held as B - 4n, the others as 4n (B =
    // q3_bias(N)).  Each inclusion-exclusion step is then one three-input add
    // (mobius3_signed), and both forms are byte addresses of the LDS table,
    // which holds t(n) at 4n and at B - 4n.  The marginal inputs come in the
    // forms that make the steps come out so: pair cells B - 4n (as the pair
    // pass writes them), single-SNP cells 4n - 4B, the class size 13B - 4n.
    // The lane's eight SNPs i: i_local = 4 (u / 2) + 2 h + u % 2, genotype a
    // in register 4 (u / 2) + 2 (u % 2) + a.
    const int i_base = ib * 16 + 2 * h;
    int pilot_best = (int)0x80000000u;  // PILOT: the lane's best screening sum
    int sb = 0;
    if constexpr (LDS) sb = screen_bound(entry_bound(tk, gthr), t.score_const, d.shift, d.tq, 81);
    #pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
        const int jm = jv[jj];
        int i_n = min(i_base, jc[jj] - 1);  // i below the middle SNP for the sub-table reads
        unsigned long long row_n = pair_row(i_n, d.M);
        unsigned long long rim = row_n + (unsigned)(m_ld[jj] - i_n - 1);
        v4u pim_n0 = pair4[2 * rim], pim_n1 = pair4[2 * rim + 1];
        #pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i_base + 4 * (u >> 1) + (u & 1);
            const int i_ld = i_n;
            const unsigned long long row_i = row_n;
            const bool valid = mv[jj] && i < jm;
            const v4u pim0 = pim_n0, pim1 = pim_n1;
            if (u + 1 < 8) {
                // next SNP's pair row, in flight while this one is scored
                i_n = min(i_base + 4 * ((u + 1) >> 1) + ((u + 1) & 1), jc[jj] - 1);
                row_n = pair_row(i_n, d.M);
                rim = row_n + (unsigned)(m_ld[jj] - i_n - 1);
                pim_n0 = pair4[2 * rim];
                pim_n1 = pair4[2 * rim + 1];
            }
            const v4u si = (single4[i_ld] << kQScaleShift) - B4;
            const unsigned long long rij = row_i + (unsigned)(jc[jj] - i_ld - 1);
            const int r0 = 4 * (u >> 1) + 2 * (u & 1);
            unsigned F[2][27];
            #pragma unroll
            for (int c = 0; c < 2; ++c) {
                const v4u pij = pair4[2 * rij + c];
                const v4u pim = c == 0 ? pim0 : pim1;
                const v4u pjm = c == 0 ? pjm0[jj] : pjm1[jj];
                #pragma unroll
                for (int a = 0; a < 2; ++a)
                    #pragma unroll
                    for (int b = 0; b < 2; ++b)
                        #pragma unroll
                        for (int e = 0; e < 2; ++e) {
                            if constexpr (PK) {
                                // 4 n(cases) + 2^T n(controls): the cases are the low
                                // T bits, the controls' 4n is the rest shifted down
                                const unsigned v = (unsigned)acc[jj][0][b][e][r0 + a];
                                F[c][9 * a + 3 * b + e] = c == 0 ? v & ((1u << T) - 1u) : (v >> (T - 2)) & ~3u;
                            } else {
                                F[c][9 * a + 3 * b + e] = (unsigned)(int)acc[jj][c][b][e][r0 + a];
                            }
                        }
                #pragma unroll
                for (int a = 0; a < 2; ++a)
                    #pragma unroll
                    for (int b = 0; b < 2; ++b) F[c][9 * a + 3 * b + 2] = pij[2 * a + b];
                #pragma unroll
                for (int a = 0; a < 2; ++a)
                    #pragma unroll
                    for (int e = 0; e < 2; ++e) F[c][9 * a + 6 + e] = pim[2 * a + e];
                #pragma unroll
                for (int b = 0; b < 2; ++b)
                    #pragma unroll
                    for (int e = 0; e < 2; ++e) F[c][18 + 3 * b + e] = pjm[2 * b + e];
                F[c][9 * 0 + 8] = si[2 * c + 0];
                F[c][9 * 1 + 8] = si[2 * c + 1];
                F[c][18 + 2] = sj[jj][2 * c + 0];
                F[c][18 + 5] = sj[jj][2 * c + 1];
                F[c][24] = sm[2 * c + 0];
                F[c][25] = sm[2 * c + 1];
                F[c][26] = nall[c];
                mobius3_signed(F[c]);
            }
            if constexpr (PILOT) {
                static_assert(LDS && !CHECK && !EMIT, "the pilot pass reads the screening table from LDS");
                if (valid) {
                    const int S = screen_sum_signed<27, REV>(F[0], F[1], B);
                    pilot_best = S > pilot_best ? S : pilot_best;
                }
                continue;
            }
            if constexpr (CHECK) {
                unsigned long long sum = 0;
                #pragma unroll
                for (int x = 0; x < 27; ++x) {
                    const unsigned n0 = (odd_twos(x) ? B - F[0][x] : F[0][x]) >> kQScaleShift;
                    const unsigned n1 = (odd_twos(x) ? B - F[1][x] : F[1][x]) >> kQScaleShift;
                    sum += (unsigned long long)n0 * cell_weight(0, x) + (unsigned long long)n1 * cell_weight(1, x);
                }
                const int cc[3] = {i, jm, m};
                digest_add(tk, valid, combo_hash<3>(cc), sum);
            }
            bool pass = valid;
            if constexpr (LDS) pass = pass && screen_sum_signed<27, REV>(F[0], F[1], B) >= sb;
            if (__ballot(pass)) {
                long long num = t.score_const;
                #pragma unroll
                for (int x = 0; x < 27; ++x) {
                    const unsigned n0 = (odd_twos(x) ? B - F[0][x] : F[0][x]) >> kQScaleShift;
                    const unsigned n1 = (odd_twos(x) ? B - F[1][x] : F[1][x]) >> kQScaleShift;
                    num += cell_term(d.tlog, (int)n0, (int)n1, (unsigned)d.N);
                }
                const unsigned long long key =
                    ((unsigned long long)i << 42) | ((unsigned long long)jm << 21) | (unsigned long long)m;
                tk_offer(tk, list, pass, num, key, gthr);
                if constexpr (LDS) sb = screen_bound(entry_bound(tk, gthr), t.score_const, d.shift, d.tq, 81);
            }
        }
    }
    if constexpr (PILOT) pilot_count(tk, t, pilot_best, 81);
}

// ---------------------------------------------------------------------------
// kGeneric: any order K.  A work item is 64 * kGenRanks consecutive colex
// ranks; lane l takes ranks l, l + 64, ...  Each lane counts all 3^K cells of
// its own combination, 27 cells (the last three SNPs) at a time for each
// genotype choice of the first K - 3 SNPs.
// ---------------------------------------------------------------------------
constexpr int kGenRanks = 4;

constexpr int pow3c(int k) { return k <= 0 ? 1 : 3 * pow3c(k - 1); }

template <int K>
EPI_DEV void colex_unrank(unsigned long long rank, int M, const unsigned long long *binom, int bstride, int (&c)[K]) {
    #pragma unroll
    for (int t = K; t >= 1; --t) {
        const unsigned long long *row = binom + (long long)t * bstride;
        int lo = t - 1, hi = M - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (row[mid] <= rank) lo = mid; else hi = mid - 1;
        }
        c[t - 1] = lo;
        rank -= row[lo];
    }
}

// The combinations of a wave's 64 consecutive colex ranks first .. first +
// 63: c enters as the combination of rank first (the same in every lane) and
// leaves as that of rank first + lane, by steps through the colex order,
// where the lowest index rises until it meets the next one, and the next
// combination then raises the lowest index that can grow and resets those
// below it to 0, 1, ...  A lane passes the loop once per run of its lowest
// index that it crosses, a few times at most.  Lanes past the last
// combination (valid false) get the first one, 0, 1, ..., K - 1.
template <int K>
EPI_DEV void colex_advance(int (&c)[K], int steps, bool valid) {
    if (!valid) {
        #pragma unroll
        for (int t = 0; t < K; ++t) c[t] = t;
        return;
    }
    #pragma unroll 1
    while (steps > 0) {
        const int room = c[1] - 1 - c[0];
        if (steps <= room) {
            c[0] += steps;
            break;
        }
        steps -= room + 1;
        int t = 1;
        #pragma unroll 1
        while (t < K - 1 && c[t] + 1 >= c[t + 1]) ++t;
        #pragma unroll
        for (int u = 0; u < K; ++u) {
            if (u == t) c[u] += 1;
            else if (u < t) c[u] = u;
        }
    }
}

// The combination after c in the colex order (wave-uniform values).
template <int K>
EPI_DEV void colex_next(int (&c)[K]) {
    int t = 0;
    #pragma unroll 1
    while (t < K - 1 && c[t] + 1 >= c[t + 1]) ++t;
    #pragma unroll
    for (int u = 0; u < K; ++u) {
        if (u == t) c[u] += 1;
        else if (u < t) c[u] = u;
    }
}

// Lane combinations of a per-combination work item, one block of 64 colex
// ranks after another: the item's first rank is unranked once, each block
// starts at the successor of the previous block's last combination, and the
// lanes step from there.
template <int K>
struct ColexWalk {
    int first[K];
    EPI_DEV void start(unsigned long long rank, int M, const unsigned long long *binom, int bstride) {
        colex_unrank<K>(rank, M, binom, bstride, first);
        #pragma unroll
        for (int t = 0; t < K; ++t) first[t] = uni(first[t]);
    }
    // this lane's combination of the block (c), then the next block's first
    EPI_DEV void lane(int (&c)[K], bool valid) {
        #pragma unroll
        for (int t = 0; t < K; ++t) c[t] = first[t];
        colex_advance<K>(c, lane_id(), valid);
        #pragma unroll
        for (int t = 0; t < K; ++t) first[t] = __builtin_amdgcn_readlane(c[t], kWave - 1);
        colex_next<K>(first);
    }
};

// Grouped counting for K >= 5: the three 27-cell chunks that differ only in
// the genotype of the last prefix SNP c[K-4] are counted in one pass over the
// words, so each word's rows and the AND of the other prefix rows are loaded
// and formed once for 81 cells instead of once per 27 (a third of the loads;
// per 32 individuals 81 AND + popcount pairs and 12 other operations).  The
// 81 class-0 counts wait for class 1 packed two to a register, so classes
// of up to 65535 individuals only.
template <int K>
EPI_DEV void g3_count(const DsView &d, const int (&c)[K], const int *dig, int cl, unsigned (&acc)[81]) {
    constexpr int NB = K - 4;
    gv4u *gm = (gv4u *)d.masks;
    const long long Mp = d.Mp;
    const int sp = c[NB];
    #pragma unroll
    for (int x = 0; x < 81; ++x) acc[x] = 0;
    const int W = d.w4[cl];
    long long off = (long long)d.wbase[cl] * 2 * Mp;
    for (int w = 0; w < W; ++w, off += 2 * Mp) {
        const v4u vm = valid_mask(d.ncls[cl], w);
        v4u X = vm;
        #pragma unroll
        for (int t = 0; t < NB; ++t) {
            const v4u r0 = gm[off + c[t]];
            const v4u r1 = gm[off + Mp + c[t]];
            X &= dig[t] == 0 ? r0 : (dig[t] == 1 ? r1 : vm & ~(r0 | r1));
        }
        const v4u p0 = gm[off + sp], p1 = gm[off + Mp + sp];
        v4u r0[3], r1[3];
        #pragma unroll
        for (int u = 0; u < 3; ++u) {
            r0[u] = gm[off + c[K - 3 + u]];
            r1[u] = gm[off + Mp + c[K - 3 + u]];
        }
        #pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned rw[3][3];
            #pragma unroll
            for (int u = 0; u < 3; ++u) {
                rw[u][0] = r0[u][q];
                rw[u][1] = r1[u][q];
                rw[u][2] = vm[q] & ~(r0[u][q] | r1[u][q]);
            }
            #pragma unroll
            for (int g = 0; g < 3; ++g) {
                const unsigned xg = X[q] & (g == 0 ? p0[q] : (g == 1 ? p1[q] : vm[q] & ~(p0[q] | p1[q])));
                #pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const unsigned xa = xg & rw[0][a];
                    #pragma unroll
                    for (int b = 0; b < 3; ++b)
                        #pragma unroll
                        for (int e = 0; e < 3; ++e)
                            acc[27 * g + 9 * a + 3 * b + e] =
                                bcnt_acc(xa & rw[1][b] & rw[2][e], acc[27 * g + 9 * a + 3 * b + e]);
                }
            }
        }
    }
}

template <int K, bool STORE, bool LDT, bool DIG>
EPI_DEV long long generic_num_g3(const DsView &d, const int (&c)[K], long long score_const, uint32_t *out,
                                 int ostride, unsigned long long *dsum) {
    constexpr int NB = K - 4;       // prefix SNPs fixed within a group
    constexpr int NG = pow3c(NB);   // groups of 81 cells
    long long num = score_const;
    #pragma unroll 1
    for (int gi = 0; gi < NG; ++gi) {
        int dig[NB > 0 ? NB : 1];
        {
            int x = gi;
            #pragma unroll
            for (int t = NB - 1; t >= 0; --t) {
                dig[t] = x % 3;
                x /= 3;
            }
        }
        unsigned acc[81], pk[41];
        g3_count<K>(d, c, dig, 0, acc);
        #pragma unroll
        for (int x = 0; x < 41; ++x) pk[x] = acc[2 * x] | (2 * x + 1 < 81 ? acc[2 * x + 1] << 16 : 0u);
        g3_count<K>(d, c, dig, 1, acc);
        #pragma unroll
        for (int x = 0; x < 81; ++x) {
            const unsigned n0 = x & 1 ? pk[x >> 1] >> 16 : pk[x >> 1] & 0xffffu;
            if constexpr (DIG)
                *dsum += (unsigned long long)n0 * cell_weight(0, gi * 81 + x) +
                         (unsigned long long)acc[x] * cell_weight(1, gi * 81 + x);
            if constexpr (STORE) {
                out[(gi * 81 + x) * ostride] = n0;
                out[(pow3c(K) + gi * 81 + x) * ostride] = acc[x];
            } else {
                num += LDT ? cell_term_lds(n0, acc[x]) : cell_term_counted(d.tlog, n0, acc[x]);
            }
        }
    }
    return num;
}

// Counts every cell of combination c, 27 (order 2: 9) at a time.  The fused
// form (STORE false) scores each chunk as it is counted and returns the
// score; with STORE the counts go to out[x * ostride] (class 0) and
// out[(3^K + x) * ostride] (class 1) instead, x the cell's index in base 3
// with the genotype of c[0] as the leading digit.  With DIG the weighted sum
// of the counts (the table part of the completeness digest) is added to
// *dsum.
template <int K, bool STORE = false, bool LDT = false, bool DIG = false>
EPI_DEV long long generic_num(const DsView &d, const int (&c)[K], long long score_const, uint32_t *out = nullptr,
                              int ostride = kWave, unsigned long long *dsum = nullptr) {
    if constexpr (K >= 5)
        if (d.ncls[0] <= 0xffff) return generic_num_g3<K, STORE, LDT, DIG>(d, c, score_const, out, ostride, dsum);
    constexpr int NPRE = K > 3 ? K - 3 : 0;
    constexpr int NCH = pow3c(NPRE);
    constexpr int L = K >= 3 ? 3 : 2;
    constexpr int CELLS = L == 3 ? 27 : 9;
    gv4u *gm = (gv4u *)d.masks;
    const long long Mp = d.Mp;
    long long num = score_const;
    for (int ch = 0; ch < NCH; ++ch) {
        int dig[NPRE > 0 ? NPRE : 1];
        {
            int x = ch;
            #pragma unroll
            for (int t = NPRE - 1; t >= 0; --t) {
                dig[t] = x % 3;
                x /= 3;
            }
        }
        unsigned acc[2][CELLS];
        #pragma unroll
        for (int cl = 0; cl < 2; ++cl) {
            #pragma unroll
            for (int x = 0; x < CELLS; ++x) acc[cl][x] = 0;
            const int W = d.w4[cl];
            long long off = (long long)d.wbase[cl] * 2 * Mp;
            for (int w = 0; w < W; ++w, off += 2 * Mp) {
                const v4u vm = valid_mask(d.ncls[cl], w);
                v4u X = vm;
                #pragma unroll
                for (int t = 0; t < NPRE; ++t) {
                    const v4u r0 = gm[off + c[t]];
                    const v4u r1 = gm[off + Mp + c[t]];
                    const v4u r2 = vm & ~(r0 | r1);
                    X &= dig[t] == 0 ? r0 : (dig[t] == 1 ? r1 : r2);
                }
                v4u rows[L][3];
                #pragma unroll
                for (int u = 0; u < L; ++u) {
                    const int s = c[K - L + u];
                    rows[u][0] = gm[off + s];
                    rows[u][1] = gm[off + Mp + s];
                    rows[u][2] = vm & ~(rows[u][0] | rows[u][1]);
                }
                #pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if constexpr (L == 3) {
                        #pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            const unsigned xa = X[q] & rows[0][a][q];
                            #pragma unroll
                            for (int b = 0; b < 3; ++b)
                                #pragma unroll
                                for (int e = 0; e < 3; ++e)
                                    acc[cl][9 * a + 3 * b + e] =
                                        bcnt_acc(xa & rows[1][b][q] & rows[2][e][q], acc[cl][9 * a + 3 * b + e]);
                        }
                    } else {
                        #pragma unroll
                        for (int a = 0; a < 3; ++a)
                            #pragma unroll
                            for (int b = 0; b < 3; ++b)
                                acc[cl][3 * a + b] = bcnt_acc(rows[0][a][q] & rows[1][b][q], acc[cl][3 * a + b]);
                    }
                }
            }
        }
        if constexpr (DIG) {
            #pragma unroll
            for (int x = 0; x < CELLS; ++x)
                *dsum += (unsigned long long)acc[0][x] * cell_weight(0, ch * CELLS + x) +
                         (unsigned long long)acc[1][x] * cell_weight(1, ch * CELLS + x);
        }
        if constexpr (STORE) {
            #pragma unroll
            for (int x = 0; x < CELLS; ++x) {
                out[(ch * CELLS + x) * ostride] = acc[0][x];
                out[(pow3c(K) + ch * CELLS + x) * ostride] = acc[1][x];
            }
        } else {
            #pragma unroll
            for (int x = 0; x < CELLS; ++x)
                num += LDT ? cell_term_lds(acc[0][x], acc[1][x]) : cell_term_counted(d.tlog, acc[0][x], acc[1][x]);
        }
    }
    return num;
}

template <int K, bool LDT, bool CHECK = false>
EPI_DEV void item_generic(const Task &t, unsigned long long local, TopK &tk, Cand *list, long long gthr,
                          const unsigned long long *binom, int bstride) {
    const DsView d = t.ds;
    const int bits = t.key_bits;
    ColexWalk<K> walk;
    walk.start(local * kGenRanks * kWave, d.M, binom, bstride);
    for (int rr = 0; rr < kGenRanks; ++rr) {
        const unsigned long long rank = (local * kGenRanks + rr) * kWave + lane_id();
        const bool valid = rank < t.n_combos;
        int c[K];
        walk.lane(c, valid);
        unsigned long long sum = 0;
        const long long num = generic_num<K, false, LDT, CHECK>(d, c, t.score_const, nullptr, kWave, &sum);
        if constexpr (CHECK) digest_add(tk, valid, combo_hash<K>(c), sum);
        unsigned long long key = 0;
        #pragma unroll
        for (int u = 0; u < K; ++u) key = (key << bits) | (unsigned long long)c[u];
        tk_offer(tk, list, valid, num, key, gthr);
    }
}

// ---------------------------------------------------------------------------
// kSeg: the segmented exploration of Section 3.4 (Algorithm 2) on a wave.  A
// block of b = 64 combinations (one per lane) first has all 2 x 3^K cells of
// its contingency tables counted, as kGeneric counts them, into the wave's
// slot of a device buffer (cell-major, 64 lanes contiguous); only then are
// the b tables read back and scored.  The item's kGenRanks blocks follow one
// another through the same slot.  A lane reads back only what it wrote, so
// program order is the only ordering needed.
// ---------------------------------------------------------------------------
template <int K, bool LDT, bool CHECK = false>
EPI_DEV void item_seg(const Task &t, unsigned long long local, TopK &tk, Cand *list, long long gthr,
                      const unsigned long long *binom, int bstride, uint32_t *slot) {
    constexpr int CELLS = pow3c(K);
    const DsView d = t.ds;
    const int bits = t.key_bits;
    const int lane = lane_id();
    uint32_t *mine = slot + lane;
    ColexWalk<K> walk;
    walk.start(local * kGenRanks * kWave, d.M, binom, bstride);
    #pragma unroll 1
    for (int rr = 0; rr < kGenRanks; ++rr) {
        const unsigned long long rank = (local * kGenRanks + rr) * kWave + lane;
        const bool valid = rank < t.n_combos;
        int c[K];
        walk.lane(c, valid);
        // phase 1: the block's tables
        (void)generic_num<K, true>(d, c, 0, mine);
        // phase 2: their scores
        long long num = t.score_const;
        unsigned long long sum = 0;
        #pragma unroll 9
        for (int x = 0; x < CELLS; ++x) {
            const unsigned n0 = mine[x * kWave], n1 = mine[(CELLS + x) * kWave];
            num += LDT ? cell_term_lds(n0, n1) : cell_term_counted(d.tlog, n0, n1);
            if constexpr (CHECK)
                sum += (unsigned long long)n0 * cell_weight(0, x) + (unsigned long long)n1 * cell_weight(1, x);
        }
        if constexpr (CHECK) digest_add(tk, valid, combo_hash<K>(c), sum);
        unsigned long long key = 0;
        #pragma unroll
        for (int u = 0; u < K; ++u) key = (key << bits) | (unsigned long long)c[u];
        tk_offer(tk, list, valid, num, key, gthr);
    }
}

// ---------------------------------------------------------------------------
// kR4: order 4 by reduced cells.  A work item is 64 * kGenRanks consecutive
// colex ranks; lane l takes ranks l, l + 64, ... (as kGeneric).  A lane counts
// the 16 cells of its combination whose four genotypes are all 0 or 1 (per 32
// individuals: 4 pair ANDs, then one three-input AND and one popcount per
// cell); every other cell follows by inclusion-exclusion from the triplet
// sub-table (written by the matrix-core kernel), the pair sub-table and the
// single-SNP counts, as for order 3; the sub-tables hold both classes of a
// cell in one register (4 n(cases) | 4 n(controls) << 16), and so do the
// lane's 81 cells.
// ---------------------------------------------------------------------------
// PILOT: the histogram-only pass (as for order 3).
template <bool LDS, bool CHECK = false, bool PILOT = false>
EPI_DEV void item_r4(const Task &t, unsigned long long local, TopK &tk, Cand *list, long long gthr,
                     const unsigned long long *binom, int bstride) {
    const DsView d = t.ds;
    int pilot_best = (int)0x80000000u;  // PILOT: the lane's best screening sum
    int sb = 0;
    if constexpr (LDS) sb = screen_bound(entry_bound(tk, gthr), t.score_const, d.shift, d.tq, 243);
    const int bits = t.key_bits;
    gv4u *gm = (gv4u *)d.masks;
    gv4u *single4 = (gv4u *)d.single;
    gv4u *pair4 = (gv4u *)t.pairs;
    gv4u *trip4 = (gv4u *)t.triples;
    const long long Mp = d.Mp;
    ColexWalk<4> walk;
    walk.start(local * kGenRanks * kWave, d.M, binom, bstride);
    #pragma unroll 1
    for (int rr = 0; rr < kGenRanks; ++rr) {
        const unsigned long long rank = (local * kGenRanks + rr) * kWave + lane_id();
        const bool valid = rank < t.n_combos;
        int c[4];
        walk.lane(c, valid);
        unsigned acc[2][16];
        // consecutive colex ranks share their two last SNPs almost always:
        // then their rows are wave-uniform scalar loads and their four
        // pairwise ANDs scalar operations, which halves the vector loads
        const int c2u = uni(c[2]), c3u = uni(c[3]);
        const bool u23 = __ballot(c[2] != c2u || c[3] != c3u) == 0ull;
        #pragma unroll
        for (int cl = 0; cl < 2; ++cl) {
            #pragma unroll
            for (int x = 0; x < 16; ++x) acc[cl][x] = 0;
            const int W = d.w4[cl];
            long long off = (long long)d.wbase[cl] * 2 * Mp;
            if (u23) {
                cv4u *sm = (cv4u *)d.masks;
                #pragma unroll 1
                for (int w = 0; w < W; ++w, off += 2 * Mp) {
                    v4u r[2][2];
                    #pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        r[u][0] = gm[off + c[u]];
                        r[u][1] = gm[off + Mp + c[u]];
                    }
                    const v4u s20 = sm[off + c2u], s21 = sm[off + Mp + c2u];
                    const v4u s30 = sm[off + c3u], s31 = sm[off + Mp + c3u];
                    #pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        unsigned p[4], y[4];
                        #pragma unroll
                        for (int ab = 0; ab < 4; ++ab) p[ab] = r[0][ab >> 1][q] & r[1][ab & 1][q];
                        y[0] = uni(s20[q] & s30[q]);
                        y[1] = uni(s20[q] & s31[q]);
                        y[2] = uni(s21[q] & s30[q]);
                        y[3] = uni(s21[q] & s31[q]);
                        #pragma unroll
                        for (int ab = 0; ab < 4; ++ab)
                            #pragma unroll
                            for (int ce = 0; ce < 4; ++ce)
                                acc[cl][4 * ab + ce] = bcnt_acc(p[ab] & y[ce], acc[cl][4 * ab + ce]);
                    }
                }
            } else {
                #pragma unroll 1
                for (int w = 0; w < W; ++w, off += 2 * Mp) {
                    v4u r[4][2];
                    #pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        r[u][0] = gm[off + c[u]];
                        r[u][1] = gm[off + Mp + c[u]];
                    }
                    #pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        unsigned p[4];
                        #pragma unroll
                        for (int ab = 0; ab < 4; ++ab) p[ab] = r[0][ab >> 1][q] & r[1][ab & 1][q];
                        #pragma unroll
                        for (int ab = 0; ab < 4; ++ab)
                            #pragma unroll
                            for (int ce = 0; ce < 4; ++ce)
                                acc[cl][4 * ab + ce] =
                                    bcnt_acc(p[ab] & r[2][ce >> 1][q] & r[3][ce & 1][q], acc[cl][4 * ab + ce]);
                    }
                }
            }
            // (keeps the scaling below out of the loop, where the compiler
            // would otherwise redo it every iteration)
            #pragma unroll
            for (int x = 0; x < 16; ++x) asm volatile("" : "+v"(acc[cl][x]));
        }
        // F[27 a + 9 b + 3 g + e]; digit 2 = marginal over that SNP, genotype
        // 2 once the inclusion-exclusion has run.  Packed cell form: a
        // register holds 4 n(cases) in its low half and 4 n(controls) in its
        // high half (classes of at most 16383 individuals), so one
        // subtraction steps both classes (no half ever goes below zero: a
        // marginal is at least the sum of its cells), and each half is the
        // byte address of its count's screening-table entry.  The
        // sub-table passes write their cells in this form.
        unsigned F[81];
        #pragma unroll
        for (int x = 0; x < 81; ++x) {
            const int a = x / 27, b = (x / 9) % 3, g = (x / 3) % 3, e = x % 3;
            if (a < 2 && b < 2 && g < 2 && e < 2) {
                const int i = 8 * a + 4 * b + 2 * g + e;
                F[x] = (acc[0][i] << kQScaleShift) | (acc[1][i] << (16 + kQScaleShift));
            }
        }
        // triplets: drop one SNP (its digit 2), cells 4a' + 2b' + d' of the rest
        #pragma unroll
        for (int drop = 0; drop < 4; ++drop) {
            int s3[3], k = 0;
            #pragma unroll
            for (int u = 0; u < 4; ++u)
                if (u != drop) s3[k++] = c[u];
            const unsigned long long tr = colex3(s3[0], s3[1], s3[2]);
            const v4u lo = trip4[2 * tr], hi = trip4[2 * tr + 1];
            #pragma unroll
            for (int y = 0; y < 8; ++y) {
                int dig[4], k2 = 0;
                #pragma unroll
                for (int u = 0; u < 4; ++u) dig[u] = u == drop ? 2 : (y >> (2 - k2++)) & 1;
                F[27 * dig[0] + 9 * dig[1] + 3 * dig[2] + dig[3]] = y < 4 ? lo[y] : hi[y - 4];
            }
        }
        // pairs: keep two SNPs
        #pragma unroll
        for (int u0 = 0; u0 < 4; ++u0)
            #pragma unroll
            for (int u1 = u0 + 1; u1 < 4; ++u1) {
                const v4u pv = pair4[colex2(c[u0], c[u1])];  // the pair sub-table in colex order
                #pragma unroll
                for (int y = 0; y < 4; ++y) {
                    int dig[4];
                    #pragma unroll
                    for (int u = 0; u < 4; ++u) dig[u] = u == u0 ? (y >> 1) : (u == u1 ? (y & 1) : 2);
                    F[27 * dig[0] + 9 * dig[1] + 3 * dig[2] + dig[3]] = pv[y];
                }
            }
        // singles and the class sizes
        #pragma unroll
        for (int u = 0; u < 4; ++u) {
            const v4u sv = single4[c[u]];
            #pragma unroll
            for (int g = 0; g < 2; ++g) {
                int dig[4];
                #pragma unroll
                for (int v = 0; v < 4; ++v) dig[v] = v == u ? g : 2;
                F[27 * dig[0] + 9 * dig[1] + 3 * dig[2] + dig[3]] =
                    (sv[g] << kQScaleShift) | (sv[2 + g] << (16 + kQScaleShift));
            }
        }
        F[80] = ((unsigned)d.ncls[0] << kQScaleShift) | ((unsigned)d.ncls[1] << (16 + kQScaleShift));
        mobius4(F);
        if constexpr (PILOT) {
            static_assert(LDS && !CHECK, "the pilot pass reads the screening table from LDS");
            if (valid) {
                const int S = screen_sum_packed<81>(F);
                pilot_best = S > pilot_best ? S : pilot_best;
            }
            continue;
        }
        if constexpr (CHECK) {
            unsigned long long sum = 0;
            #pragma unroll
            for (int x = 0; x < 81; ++x)
                sum += (unsigned long long)((F[x] & 0xffffu) >> kQScaleShift) * cell_weight(0, x) +
                       (unsigned long long)(F[x] >> (16 + kQScaleShift)) * cell_weight(1, x);
            digest_add(tk, valid, combo_hash<4>(c), sum);
        }
        bool pass = valid;
        if constexpr (LDS) pass = pass && screen_sum_packed<81>(F) >= sb;
        if (__ballot(pass)) {
            long long num = t.score_const;
            #pragma unroll
            for (int x = 0; x < 81; ++x)
                num += cell_term_counted(d.tlog, (F[x] & 0xffffu) >> kQScaleShift, F[x] >> (16 + kQScaleShift));
            unsigned long long key = 0;
            #pragma unroll
            for (int u = 0; u < 4; ++u) key = (key << bits) | (unsigned long long)c[u];
            tk_offer(tk, list, pass, num, key, gthr);
            if constexpr (LDS) sb = screen_bound(entry_bound(tk, gthr), t.score_const, d.shift, d.tq, 243);
        }
    }
    if constexpr (PILOT) pilot_count(tk, t, pilot_best, 243);
}

// ---------------------------------------------------------------------------
// Persistent scan kernel: four independent waves per workgroup.  The
// workgroup pops chunks of work items from a device queue that runs over the
// concatenated item spaces of all tasks of the launch, in task order; each
// wave keeps its own best-K list and prefix-row slot in LDS.
// ---------------------------------------------------------------------------
// Register budget per instantiation: enough waves per SIMD to hide load
// latency; the accumulators (16 per prefix for order 3, 8 for order 2, 128
// for the matrix-core order-3 kernels: two classes of one middle SNP, or one
// accumulator for both classes of each of two; 128 for order 2 on the
// matrix cores too) set the floor.
template <int NP2, int NP3, int GK>
constexpr int scan_waves_per_eu() {
    return NP3 == kNpMfma2 || NP2 == kNpMfma ? 2
                           : (GK >= 4 ? 2 : (GK == 3 ? 3 : (NP3 >= 8 ? 2 : (NP3 >= 4 ? 3 : (NP3 >= 2 ? 4 : (NP2 >= 8 ? 3 : 4))))));
}

// Items of a task's pilot pass: pilot_n consecutive ones from pilot_first.
EPI_DEV bool is_pilot_item(const Task &t, unsigned long long local) {
    return local >= t.pilot_first && local - t.pilot_first < (unsigned long long)t.pilot_n;
}

// CHECK: the checking instantiation, which also adds every scored
// combination to its task's completeness digest (the same results otherwise).
template <int NP2, int NP3, int GK, bool CHECK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(scan_waves_per_eu<NP2, NP3, GK>())))
scan_persistent(const Task *__restrict__ tasks, int n_tasks, unsigned long long total_items,
                unsigned long long *__restrict__ queue, const unsigned long long *__restrict__ binom, int bstride,
                int tab_cap, int kmax, int stage_cap) {
    // dynamic LDS (the kernel has no static LDS, so the screening table
    // starts at LDS address 0 and a count's byte offset is its address):
    //   [tab_cap floats: screening table of the current dataset]
    //   [4 x kmax best-K lists][4 x stage_cap uint4: staged rows][2 x u64: queue chunk]
    extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
    unsigned *s_tab = (unsigned *)s_dyn;
    const int wave = uni((int)(threadIdx.x >> 6));  // wave index in the workgroup (uniform per wave)
    const long long lists_off = ((long long)tab_cap * 4 + 15) & ~15LL;
    const long long stage_off = lists_off + (long long)4 * kmax * sizeof(Cand);
    Cand *s_list = (Cand *)(s_dyn + lists_off) + wave * kmax;
    v4u *s_stage = (v4u *)(s_dyn + stage_off) + wave * stage_cap;
    unsigned long long *s_chunk = (unsigned long long *)(s_dyn + stage_off + (long long)4 * stage_cap * sizeof(v4u));
    TopK tk;
    tk.n = 0;
    tk.K = 1;
    tk.cap = kmax;
    tk.wi = 0;
    tk.wn = 0;
    tk.wk = 0;
    tk.hist = nullptr;
    tk.added = 0;
    tk.top = -1;
    tk.dsum = 0;
    tk.dn = 0;
    tk.nohist = 0;
    int cur = -1;
    long long gthr = (long long)0x8000000000000000ull;
    const uint32_t *loaded = nullptr;  // dataset whose screening table is in s_tab
    bool loaded_rev = false;           // both halves of it (else the first)
    // Guided self-scheduling, one queue atomic per chunk of 4 x `per` items for
    // the whole workgroup; the chunk shrinks with the remaining work (estimated
    // from the last chunk).  Wave w takes items first + w, first + w + 4, ...
    const unsigned long long n_waves = (unsigned long long)gridDim.x * 4;
    unsigned long long est = 0;
    #pragma unroll 1
    for (;;) {
        if (threadIdx.x == 0) {
            unsigned long long per = (total_items - min(est, total_items)) / (2 * n_waves);
            per = per < 1 ? 1 : (per > 32 ? 32 : per);
            s_chunk[0] = atomicAdd(queue, 4 * per);
            s_chunk[1] = per;
        }
        __syncthreads();
        // values read back from LDS are wave-uniform: keep them in SGPRs
        const unsigned long long first = rfl64(s_chunk[0]), per = rfl64(s_chunk[1]);
        __syncthreads();
        if (first >= total_items) break;
        const unsigned long long end = min(first + 4 * per, total_items);
        est = end;
        // the chunk's dataset takes the LDS screening table if it fits
        {
            int lo = 0, hi = n_tasks - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (tasks[mid].item_base <= first) lo = mid; else hi = mid - 1;
            }
            const Task &T0 = tasks[lo];
            // the screening reads address the table from LDS address 0; the
            // mirrored half too for the kernels in the signed cell form, when
            // it fits
            const int ent_fwd = T0.ds.N + 1, ent_rev = 2 * T0.ds.N + 2;
            const bool want = (T0.variant == kF2 || T0.variant == kF2Fold || T0.variant == kF3 || T0.variant == kR4) &&
                              ent_fwd <= tab_cap &&
                              (unsigned)(uintptr_t)(lu32 *)s_tab == 0u;
            const bool sgn = T0.variant == kF3 && is_mfma_np(T0.np);
            const bool rev = want && sgn && ent_rev <= tab_cap;  // read only in the signed cell form
            if (want && (loaded != T0.ds.itab || (rev && !loaded_rev))) {
                const int ent = rev ? ent_rev : ent_fwd;
                #pragma unroll 1
                for (int x = threadIdx.x; x < ent; x += blockDim.x) s_tab[x] = T0.ds.itab[x];
                __syncthreads();
                loaded = T0.ds.itab;
                loaded_rev = rev;
            }
            // the per-combination kernels: the exact n ln n table, n <= N
            const int ent_tl = 2 * (T0.ds.N + 1);
            const bool want_tl = (T0.variant == kGeneric || T0.variant == kSeg) && ent_tl <= tab_cap &&
                                 (unsigned)(uintptr_t)(lu32 *)s_tab == 0u;
            if (want_tl && loaded != (const uint32_t *)T0.ds.tlog) {
                const uint32_t *src = (const uint32_t *)T0.ds.tlog;
                #pragma unroll 1
                for (int x = threadIdx.x; x < ent_tl; x += blockDim.x) s_tab[x] = src[x];
                __syncthreads();
                loaded = src;
                loaded_rev = false;
            }
        }
        #pragma unroll 1
        for (unsigned long long item = first + wave; item < end; item += 4) {
            int lo = 0, hi = n_tasks - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (tasks[mid].item_base <= item) lo = mid; else hi = mid - 1;
            }
            if (lo != cur) {
                if (cur >= 0 && !is_emit(tasks[cur].variant)) {
                    if (tk.n == tk.K && tk.wn > gthr && lane_id() == 0) atomicMax(tasks[cur].thr, bias(tk.wn));
                    tk_flush(tk, s_list, tasks[cur]);
                    if constexpr (CHECK) digest_flush(tk, tasks[cur]);
                }
                cur = lo;
                tk.n = 0;
                tk.K = tasks[cur].top_k;
                tk.hist = is_emit(tasks[cur].variant) ? nullptr : tasks[cur].hist;
                tk.added = 0;
                tk.top = -1;
                gthr = (long long)0x8000000000000000ull;
                if (!is_emit(tasks[cur].variant)) {
                    // a new task starts from the bound published so far
                    long long g = 0;
                    if (lane_id() == 0) g = load_thr(tasks[cur].thr);
                    gthr = (long long)rfl64((unsigned long long)g);
                }
            }
            const Task &T = tasks[cur];
            // the bound other waves have published: read before every item,
            // taken up after it (the item's own waits cover the load)
            long long g_pub = (long long)0x8000000000000000ull;
            if (!is_emit(T.variant) && lane_id() == 0) g_pub = load_thr(T.thr);
            const unsigned long long local = item - T.item_base + T.first_item;
            const bool lds = loaded != nullptr && T.ds.itab == loaded;
            const bool ldt = loaded != nullptr && (const uint32_t *)T.ds.tlog == loaded;
            // the pilot pass has counted the combinations of its items
            tk.nohist = is_pilot_item(T, local);
            switch (T.variant) {
            case kF2:
                if constexpr (NP2 == kNpMfma) {
                    if (lds) item_f2m<true, CHECK>(T, local, tk, s_list, gthr);
                    else item_f2m<false, CHECK>(T, local, tk, s_list, gthr);
                } else if constexpr (NP2 > 0) {
                    if (lds) item_f2<NP2, false, true, true, CHECK>(T, local, tk, s_list, gthr, s_stage, stage_cap);
                    else item_f2<NP2, false, false, true, CHECK>(T, local, tk, s_list, gthr, s_stage, stage_cap);
                }
                break;
            case kF2Emit:
                if constexpr (NP2 > 0 && NP2 != kNpMfma)
                    item_f2<NP2, true, false>(T, local, tk, s_list, gthr, s_stage, stage_cap);
                break;
            case kF2Fold:
                if constexpr (NP2 > 0 && NP2 != kNpMfma) {
                    if (lds) item_f2<NP2, true, true, true, CHECK>(T, local, tk, s_list, gthr, s_stage, stage_cap);
                    else item_f2<NP2, true, false, true, CHECK>(T, local, tk, s_list, gthr, s_stage, stage_cap);
                }
                break;
            case kF3Emit:
                if constexpr (NP3 == kNpMfma) item_f3m<false, false, false, true>(T, local, tk, s_list, gthr, s_stage);
                break;
            case kR4:
                if constexpr (GK == 4) {
                    if (lds) item_r4<true, CHECK>(T, local, tk, s_list, gthr, binom, bstride);
                    else item_r4<false, CHECK>(T, local, tk, s_list, gthr, binom, bstride);
                }
                break;
            case kF3:
                if constexpr (is_mfma_np(NP3)) {
                    constexpr bool i8 = NP3 == kNpMfmaI8;
                    constexpr int nj = NP3 == kNpMfma2 ? 2 : 1;
                    if (lds && loaded_rev)
                        item_f3m<true, true, i8, false, CHECK, nj>(T, local, tk, s_list, gthr, s_stage);
                    else if (lds) item_f3m<true, false, i8, false, CHECK, nj>(T, local, tk, s_list, gthr, s_stage);
                    else item_f3m<false, false, i8, false, CHECK, nj>(T, local, tk, s_list, gthr, s_stage);
                } else if constexpr (NP3 > 0) {
                    if (lds) item_f3<NP3, true, CHECK>(T, local, tk, s_list, gthr, s_stage, stage_cap);
                    else item_f3<NP3, false, CHECK>(T, local, tk, s_list, gthr, s_stage, stage_cap);
                }
                break;
            case kSeg:
                if constexpr (GK > kSegGk) {
                    uint32_t *slot = T.seg + (size_t)(blockIdx.x * 4 + wave) * (2 * kWave * pow3c(GK - kSegGk));
                    if (ldt) item_seg<GK - kSegGk, true, CHECK>(T, local, tk, s_list, gthr, binom, bstride, slot);
                    else item_seg<GK - kSegGk, false, CHECK>(T, local, tk, s_list, gthr, binom, bstride, slot);
                }
                break;
            default:
                if constexpr (GK > 0 && GK < kSegGk) {
                    if (ldt) item_generic<GK, true, CHECK>(T, local, tk, s_list, gthr, binom, bstride);
                    else item_generic<GK, false, CHECK>(T, local, tk, s_list, gthr, binom, bstride);
                }
                break;
            }
            if (!is_emit(T.variant)) {
                const long long g = (long long)rfl64((unsigned long long)g_pub);
                gthr = g > gthr ? g : gthr;
            }
            if (tk.added) {
                // combinations were counted: raise and publish the bound
                tk.added = 0;
                const long long hb = hist_bound(tk.hist, tk.K, tk.top);
                if (hb > gthr) {
                    gthr = hb;
                    if (lane_id() == 0) atomicMax(T.thr, bias(hb));
                }
            }
        }
        if (cur >= 0 && !is_emit(tasks[cur].variant) && tk.n == tk.K && tk.wn > gthr) {
            if (lane_id() == 0) atomicMax(tasks[cur].thr, bias(tk.wn));
            gthr = tk.wn;
        }
    }
    if (cur >= 0 && !is_emit(tasks[cur].variant)) {
        tk_flush(tk, s_list, tasks[cur]);
        if constexpr (CHECK) digest_flush(tk, tasks[cur]);
    }
}

typedef void (*ScanKernelFn)(const Task *, int, unsigned long long, unsigned long long *, const unsigned long long *,
                             int, int, int, int);

struct ScanKernelEntry {
    int np2, np3, gk;
    ScanKernelFn fn;
};

// Every instantiation of the scan kernel, in one table per CHECK value: this
// file is compiled twice, once as is (everything but the checking
// instantiations) and once with EPI_SCAN_CHECK defined (only those), so the
// two large sets of instantiations compile in parallel.
#define EPI_SCAN_KERNELS(CK)                                                                                     \
    {2, 0, 0, scan_persistent<2, 0, 0, CK>}, {4, 0, 0, scan_persistent<4, 0, 0, CK>},                             \
        {8, 0, 0, scan_persistent<8, 0, 0, CK>}, /* order 2 / pair sub-table */                                  \
        {kNpMfma, 0, 0, scan_persistent<kNpMfma, 0, 0, CK>}, /* order 2, matrix cores */                         \
        {0, 1, 0, scan_persistent<0, 1, 0, CK>}, {0, 2, 0, scan_persistent<0, 2, 0, CK>},                         \
        {0, 4, 0, scan_persistent<0, 4, 0, CK>}, {0, 8, 0, scan_persistent<0, 8, 0, CK>}, /* order 3 */          \
        {0, 0, 4, scan_persistent<0, 0, 4, CK>}, {0, 0, 5, scan_persistent<0, 0, 5, CK>}, /* per combination */ \
        {0, 0, 6, scan_persistent<0, 0, 6, CK>}, {0, 0, 7, scan_persistent<0, 0, 7, CK>},                         \
        {0, 0, 8, scan_persistent<0, 0, 8, CK>},                                                                   \
        {0, 0, kSegGk + 2, scan_persistent<0, 0, kSegGk + 2, CK>}, /* segmented (two-phase) */                   \
        {0, 0, kSegGk + 3, scan_persistent<0, 0, kSegGk + 3, CK>},                                                 \
        {0, 0, kSegGk + 4, scan_persistent<0, 0, kSegGk + 4, CK>},                                                 \
        {0, 0, kSegGk + 5, scan_persistent<0, 0, kSegGk + 5, CK>},                                                 \
        {0, 0, kSegGk + 6, scan_persistent<0, 0, kSegGk + 6, CK>},                                                 \
        {0, 0, kSegGk + 7, scan_persistent<0, 0, kSegGk + 7, CK>},                                                 \
        {0, 0, kSegGk + 8, scan_persistent<0, 0, kSegGk + 8, CK>},                                                 \
        {0, kNpMfma, 0, scan_persistent<0, kNpMfma, 0, CK>}, /* order 3, matrix cores */                         \
        {0, kNpMfmaI8, 0, scan_persistent<0, kNpMfmaI8, 0, CK>},                                                  \
        {0, kNpMfma2, 0, scan_persistent<0, kNpMfma2, 0, CK>},

#ifdef EPI_SCAN_CHECK
static const ScanKernelEntry kScanKernelsCheck[] = {EPI_SCAN_KERNELS(true)};

ScanKernelFn find_scan_kernel_check(int np2, int np3, int gk) {
    for (const auto &e : kScanKernelsCheck)
        if (e.np2 == np2 && e.np3 == np3 && e.gk == gk) return e.fn;
    return nullptr;
}
#else
// ---------------------------------------------------------------------------
// Pilot pass of the matrix-core order-3 and reduced-cell order-4 scans of a
// launch group, launched before its main launch.  Each task with pilot_n > 0
// has pilot_n consecutive pilot items (from the middle of its scan, sharing
// operand blocks in L2 as the main launch's items do), numbered from
// pilot_base in the pilot launch; a workgroup takes 4 of them (one per wave,
// never two tasks).  A wave passes over its item counting the best lower
// bound of its scores into the task's histogram (one count); the last wave of
// a task reads the bound the histogram gives (the K-th best of lower bounds
// of distinct combinations is at most the task's final K-th best) and
// publishes it.  Every wave of the main launch starts from that bound, and
// the main launch does not count the pilot items again.  Same launch shape
// and LDS layout as the scan kernel.
// ---------------------------------------------------------------------------
template <int NP2, int NP3, int GK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(scan_waves_per_eu<NP2, NP3, GK>())))
scan_pilot(const Task *__restrict__ tasks, int n_tasks, unsigned long long total, const unsigned long long *binom,
           int bstride, int tab_cap, int kmax, int stage_cap) {
    extern __shared__ __attribute__((aligned(16))) unsigned char s_dyn[];
    unsigned *s_tab = (unsigned *)s_dyn;
    // the screening reads address the table from LDS address 0
    if ((unsigned)(uintptr_t)(lu32 *)s_tab != 0u) return;
    const int wave = uni((int)(threadIdx.x >> 6));
    const long long lists_off = ((long long)tab_cap * 4 + 15) & ~15LL;
    const long long stage_off = lists_off + (long long)4 * kmax * sizeof(Cand);
    Cand *s_list = (Cand *)(s_dyn + lists_off) + wave * kmax;
    v4u *s_stage = (v4u *)(s_dyn + stage_off) + wave * stage_cap;
    TopK tk;
    tk.n = 0;
    tk.K = 1;
    tk.cap = kmax;
    tk.wi = 0;
    tk.wn = 0;
    tk.wk = 0;
    tk.hist = nullptr;
    tk.added = 0;
    tk.top = -1;
    tk.dsum = 0;
    tk.dn = 0;
    tk.nohist = 0;
    constexpr bool i8 = NP3 == kNpMfmaI8;
    constexpr int nj = NP3 == kNpMfma2 ? 2 : 1;
    const long long none = (long long)0x8000000000000000ull;
    const uint32_t *loaded = nullptr;
    bool loaded_rev = false;
    #pragma unroll 1
    for (unsigned long long g = (unsigned long long)blockIdx.x * 4; g < total; g += (unsigned long long)gridDim.x * 4) {
        int lo = 0, hi = n_tasks - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tasks[mid].pilot_base <= g) lo = mid; else hi = mid - 1;
        }
        const Task &T = tasks[lo];
        // the task's screening table (the host takes only tasks whose table
        // fits), with its mirrored half for the signed cell form of order 3
        const int ent_fwd = T.ds.N + 1, ent_rev = 2 * T.ds.N + 2;
        const bool rev = NP3 != 0 && ent_rev <= tab_cap;
        if (ent_fwd <= tab_cap && (loaded != T.ds.itab || (rev && !loaded_rev))) {
            __syncthreads();  // every wave is done with the previous table
            const int ent = rev ? ent_rev : ent_fwd;
            #pragma unroll 1
            for (int x = threadIdx.x; x < ent; x += blockDim.x) s_tab[x] = T.ds.itab[x];
            __syncthreads();
            loaded = T.ds.itab;
            loaded_rev = rev;
        }
        const unsigned long long local = T.pilot_first + (g - T.pilot_base) + (unsigned long long)wave;
        tk.hist = T.hist;
        tk.K = T.top_k;
        tk.top = -1;
        tk.added = 0;
        if (ent_fwd <= tab_cap && local < T.n_items) {
            if constexpr (GK == 4) {
                item_r4<true, false, true>(T, local, tk, s_list, none, binom, bstride);
            } else if constexpr (NP2 == kNpMfma) {
                item_f2m<true, false, true>(T, local, tk, s_list, none);
            } else if constexpr (NP2 > 0) {
                item_f2<NP2, false, true, true, false, true>(T, local, tk, s_list, none, s_stage, stage_cap);
            } else {
                if (rev) item_f3m<true, true, i8, false, false, nj, true>(T, local, tk, s_list, none, s_stage);
                else item_f3m<true, false, i8, false, false, nj, true>(T, local, tk, s_list, none, s_stage);
            }
        }
        // the task's last pilot wave takes the bound (from one octave above
        // its own count down)
        __threadfence();
        unsigned prev = 0;
        if (lane_id() == 0) prev = atomicAdd(T.hist + kPilotWord, 1u);
        prev = (unsigned)__builtin_amdgcn_readfirstlane((int)prev);
        if (prev + 1 == (unsigned)T.pilot_n && tk.top >= 0) {
            __threadfence();
            const long long hb = hist_bound(T.hist, T.top_k, tk.top);
            if (hb != none && lane_id() == 0) atomicMax(T.thr, bias(hb));
        }
    }
}

// ---------------------------------------------------------------------------
// Best-K selection over a task's candidate buffer: one 1024-thread workgroup
// per task; candidates below the task's final threshold are dropped, the rest
// are bitonic-sorted in LDS (best first) chunk by chunk.
// ---------------------------------------------------------------------------
EPI_DEV void bitonic_sort_best_first(Cand *buf, int P) {
    for (int k = 2; k <= P; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int ixj = i ^ jj;
                if (ixj > i) {
                    const Cand a = buf[i], b = buf[ixj];
                    const bool up = (i & k) == 0;
                    const bool sw = up ? better(b.num, b.key, a.num, a.key) : better(a.num, a.key, b.num, b.key);
                    if (sw) {
                        buf[i] = b;
                        buf[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Best K of src[lo, hi) (entries below g dropped) into out[0, K), best first.
EPI_DEV void merge_range(const Cand *src, unsigned lo, unsigned hi, long long g, int K, Cand *buf, int *s_ctr,
                         Cand *out) {
    const Cand sentinel{(long long)0x8000000000000000ull, ~0ull};
    for (int i = threadIdx.x; i < kMergeSlots; i += blockDim.x) buf[i] = sentinel;
    __syncthreads();
    int fill = K;
    for (unsigned base = lo; base < hi; base += blockDim.x) {
        const unsigned i = base + threadIdx.x;
        Cand c = sentinel;
        bool keep = false;
        if (i < hi) {
            c = src[i];
            keep = c.num >= g;
        }
        const int n = __syncthreads_count(keep);
        if (fill + n > kMergeSlots) {
            int P = 64;
            while (P < fill) P <<= 1;
            bitonic_sort_best_first(buf, P);
            for (int x = K + threadIdx.x; x < kMergeSlots; x += blockDim.x) buf[x] = sentinel;
            fill = K;
            __syncthreads();
        }
        if (threadIdx.x == 0) *s_ctr = fill;
        __syncthreads();
        if (keep) buf[atomicAdd(s_ctr, 1)] = c;
        __syncthreads();
        fill += n;
    }
    int P = 64;
    while (P < fill) P <<= 1;
    bitonic_sort_best_first(buf, P);
    for (int r = threadIdx.x; r < K; r += blockDim.x) out[r] = buf[r];
}

// Stage 1: workgroup (part, task) reduces its slice of the task's candidate
// buffer to the best K.
__global__ void __launch_bounds__(1024) merge_part_kernel(const Task *__restrict__ tasks, Cand *__restrict__ parts) {
    __shared__ Cand buf[kMergeSlots];
    __shared__ int s_ctr;
    const Task &t = tasks[blockIdx.y];
    unsigned count = *t.cand_count;
    count = count < t.cand_cap ? count : t.cand_cap;
    const unsigned lo = (unsigned)((unsigned long long)count * blockIdx.x / gridDim.x);
    const unsigned hi = (unsigned)((unsigned long long)count * (blockIdx.x + 1) / gridDim.x);
    merge_range(t.cand, lo, hi, load_thr(t.thr), t.top_k, buf, &s_ctr,
                parts + ((long long)blockIdx.y * gridDim.x + blockIdx.x) * kMaxTopK);
}

// Stage 2: one workgroup per task merges the stage-1 lists.
__global__ void __launch_bounds__(1024) merge_final_kernel(const Task *__restrict__ tasks, const Cand *__restrict__ parts,
                                                           int n_parts, Cand *__restrict__ results) {
    __shared__ Cand buf[kMergeSlots];
    __shared__ int s_ctr;
    const Task &t = tasks[blockIdx.x];
    const int K = t.top_k;
    const Cand *src = parts + (long long)blockIdx.x * n_parts * kMaxTopK;
    // gather the n_parts lists (K entries each, stride kMaxTopK) behind the best K
    const Cand sentinel{(long long)0x8000000000000000ull, ~0ull};
    for (int i = threadIdx.x; i < kMergeSlots; i += blockDim.x) buf[i] = sentinel;
    __syncthreads();
    const long long g = load_thr(t.thr);
    int fill = K;
    if (K + n_parts * K <= kMergeSlots) {
        // all lists at once, every load in flight together; only entries
        // that reach the task's bound are kept, packed behind the first K
        // slots, so the sort covers those alone
        if (threadIdx.x == 0) s_ctr = K;
        __syncthreads();
        for (int i = threadIdx.x; i < n_parts * K; i += blockDim.x) {
            const int p = i / K, r = i - p * K;
            const Cand c = src[(long long)p * kMaxTopK + r];
            if (c.num >= g) buf[atomicAdd(&s_ctr, 1)] = c;
        }
        __syncthreads();
        fill = s_ctr;
    } else
    for (int p = 0; p < n_parts; ++p) {
        if (fill + K > kMergeSlots) {
            int P = 64;
            while (P < fill) P <<= 1;
            bitonic_sort_best_first(buf, P);
            for (int x = K + threadIdx.x; x < kMergeSlots; x += blockDim.x) buf[x] = sentinel;
            fill = K;
            __syncthreads();
        }
        for (int r = threadIdx.x; r < K; r += blockDim.x) {
            const Cand c = src[(long long)p * kMaxTopK + r];
            buf[fill + r] = c.num >= g ? c : sentinel;
        }
        __syncthreads();
        fill += K;
    }
    int P = 64;
    while (P < fill) P <<= 1;
    bitonic_sort_best_first(buf, P);
    for (int r = threadIdx.x; r < K; r += blockDim.x) results[(long long)blockIdx.x * kMaxTopK + r] = buf[r];
}

// ---------------------------------------------------------------------------
// Result tables: one wave per (task, result).  Decodes the combination,
// converts the score, and counts the full 2 x 3^k table straight from the
// masks (genotype-2 rows = valid & ~(row0 | row1)).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) finalize_kernel(const Task *__restrict__ tasks, const Cand *__restrict__ results,
                                                      const ResultLayout *__restrict__ layout, char *__restrict__ out) {
    const int ti = blockIdx.y;
    const int r = blockIdx.x;
    const Task &t = tasks[ti];
    const int K = t.top_k;
    if (r >= K) return;
    const int k = t.order;
    const DsView d = t.ds;
    char *blk = out + layout[ti].offset;
    int32_t *hdr = (int32_t *)blk;
    int32_t *combos = (int32_t *)(blk + 16);
    float *scores = (float *)(blk + 16 + (long long)K * k * 4);
    uint32_t *tables = (uint32_t *)(blk + 16 + (long long)K * k * 4 + (long long)K * 4);
    const Cand *res = results + (long long)ti * kMaxTopK;
    const unsigned long long sentinel_key = ~0ull;
    if (r == 0) {
        int nv = 0;
        for (int x = threadIdx.x; x < K; x += kWave) nv += res[x].key != sentinel_key ? 1 : 0;
        #pragma unroll
        for (int off = 32; off > 0; off >>= 1) nv += __shfl_xor(nv, off);
        if (threadIdx.x == 0) {
            hdr[0] = nv;
            hdr[1] = *d.err;  // nonzero: the dataset's last packing had invalid input
        }
    }
    const Cand e = res[r];
    if (e.key == sentinel_key) return;
    const int bits = t.key_bits;
    const unsigned long long kmask = (1ull << bits) - 1ull;
    int c[kMaxBinomOrder];
    for (int u = 0; u < k; ++u) c[u] = min((int)((e.key >> (bits * (k - 1 - u))) & kmask), d.Mp - 1);
    if (threadIdx.x < k) combos[r * k + threadIdx.x] = c[threadIdx.x];
    if (threadIdx.x == 0) scores[r] = (float)(ldexp((double)e.num, -d.shift) / (double)d.N);
    int cells = 1;
    for (int u = 0; u < k; ++u) cells *= 3;
    gv4u *gm = (gv4u *)d.masks;
    const long long Mp = d.Mp;
    if (cells <= 32) {
        // orders 2-3: lanes that share a cell take every parts-th word of
        // it, and their counts meet in LDS
        __shared__ unsigned s_cnt[2][32];
        const int parts = kWave / cells;
        s_cnt[threadIdx.x >> 5][threadIdx.x & 31] = 0;
        __syncthreads();
        const int x = threadIdx.x % cells, part = threadIdx.x / cells;
        if (part < parts) {
            int g[3];
            for (int u = k - 1, y = x; u >= 0; --u) {
                g[u] = y % 3;
                y /= 3;
            }
            for (int cl = 0; cl < 2; ++cl) {
                unsigned cnt = 0;
                #pragma unroll 2
                for (int w = part; w < d.w4[cl]; w += parts) {
                    const long long off = ((long long)d.wbase[cl] + w) * 2 * Mp;
                    const v4u vm = valid_mask(d.ncls[cl], w);
                    v4u X = vm;
                    for (int u = 0; u < k; ++u) {
                        const v4u r0 = gm[off + c[u]];
                        const v4u r1 = gm[off + Mp + c[u]];
                        X &= g[u] == 0 ? r0 : (g[u] == 1 ? r1 : (vm & ~(r0 | r1)));
                    }
                    cnt += __builtin_popcount(X[0]) + __builtin_popcount(X[1]) + __builtin_popcount(X[2]) +
                           __builtin_popcount(X[3]);
                }
                atomicAdd(&s_cnt[cl][x], cnt);
            }
        }
        __syncthreads();
        if (threadIdx.x < cells)
            for (int cl = 0; cl < 2; ++cl) tables[((long long)r * 2 + cl) * cells + threadIdx.x] = s_cnt[cl][threadIdx.x];
        return;
    }
    for (int x = threadIdx.x; x < cells; x += kWave) {
        int g[kMaxBinomOrder];
        int y = x;
        for (int u = k - 1; u >= 0; --u) {
            g[u] = y % 3;
            y /= 3;
        }
        for (int cl = 0; cl < 2; ++cl) {
            unsigned cnt = 0;
            long long off = (long long)d.wbase[cl] * 2 * Mp;
            for (int w = 0; w < d.w4[cl]; ++w, off += 2 * Mp) {
                const v4u vm = valid_mask(d.ncls[cl], w);
                v4u X = vm;
                for (int u = 0; u < k; ++u) {
                    const v4u r0 = gm[off + c[u]];
                    const v4u r1 = gm[off + Mp + c[u]];
                    X &= g[u] == 0 ? r0 : (g[u] == 1 ? r1 : (vm & ~(r0 | r1)));
                }
                cnt += __builtin_popcount(X[0]) + __builtin_popcount(X[1]) + __builtin_popcount(X[2]) +
                       __builtin_popcount(X[3]);
            }
            tables[((long long)r * 2 + cl) * cells + x] = cnt;
        }
    }
}

// ---------------------------------------------------------------------------
// The three steps of Section 2 as separate passes over a list of
// combinations (n x K int32 SNP indices): genotype tables (Section 2.1),
// contingency tables (Section 2.2) and mutual information (Section 2.3,
// Equation 1).  An index outside [0, M) or a table that does not fit the
// dataset sets *err and leaves that combination's output unwritten (tables,
// rows) or NaN (MI).
// ---------------------------------------------------------------------------

// Genotype rows, depth-first over the genotypes of SNPs T .. K-1: p is the
// AND of the rows chosen for SNPs 0 .. T-1 (Algorithm 1's combine step adds
// one SNP per level); leaves are written W words apart.
template <int T, int K>
EPI_DEV void gt_walk(const unsigned (&r)[K][3], unsigned p, uint32_t *&o, int W) {
    if constexpr (T + 2 >= K) {
        #pragma unroll
        for (int g = 0; g < 3; ++g) {
            const unsigned q = p & r[T][g];
            if constexpr (T + 1 == K) {
                *o = q;
                o += W;
            } else {
                gt_walk<T + 1, K>(r, q, o, W);
            }
        }
    } else {
        #pragma unroll 1
        for (int g = 0; g < 3; ++g) {
            const unsigned rg = g == 0 ? r[T][0] : (g == 1 ? r[T][1] : r[T][2]);
            gt_walk<T + 1, K>(r, p & rg, o, W);
        }
    }
}

// Leading SNPs whose genotypes split a combination's rows over threads.
template <int K>
constexpr int gt_split() { return K >= 5 ? 2 : 0; }

// One thread per (combination, genotypes of its first gt_split SNPs, 32-bit
// word of the two classes' rows): rows [i][x][w], W = 4 (w4[0] + w4[1])
// words, class 0 first.
template <int K>
__global__ void __launch_bounds__(256) gt_kernel(DsView d, const int32_t *__restrict__ combos, unsigned long long n,
                                                 uint32_t *__restrict__ rows, int *__restrict__ err) {
    constexpr int P = pow3c(K), S = gt_split<K>(), PS = pow3c(S);
    const int W0 = 4 * d.w4[0], W = W0 + 4 * d.w4[1];
    const unsigned *m = (const unsigned *)d.masks;
    const long long Mp = d.Mp;
    const unsigned long long total = n * PS * (unsigned long long)W;
    for (unsigned long long id = blockIdx.x * 256ull + threadIdx.x; id < total;
         id += (unsigned long long)gridDim.x * 256ull) {
        const unsigned long long rest = id / (unsigned)W;
        const int w = (int)(id - rest * (unsigned)W);
        const unsigned long long i = rest / PS;
        const int sub = (int)(rest - i * PS);
        const int cl = w < W0 ? 0 : 1;
        const int wc = w - (cl ? W0 : 0);
        const long long g4 = d.wbase[cl] + wc / 4;
        const int left = d.ncls[cl] - 32 * wc;
        const unsigned vm = left >= 32 ? ~0u : (left <= 0 ? 0u : ((1u << left) - 1u));
        unsigned r[K][3];
        bool bad = false;
        #pragma unroll
        for (int t = 0; t < K; ++t) {
            int sn = combos[i * K + t];
            bad |= sn < 0 || sn >= d.M;
            sn = sn < 0 || sn >= d.M ? 0 : sn;
            r[t][0] = m[((g4 * 2 + 0) * Mp + sn) * 4 + (wc & 3)];
            r[t][1] = m[((g4 * 2 + 1) * Mp + sn) * 4 + (wc & 3)];
            r[t][2] = vm & ~(r[t][0] | r[t][1]);
        }
        if (bad) {
            atomicOr(err, 1);
            continue;
        }
        unsigned p = ~0u;
        #pragma unroll
        for (int t = 0, x = sub, div = PS / 3; t < S; ++t, div /= 3) {
            const int g = x / div;
            x -= g * div;
            p &= g == 0 ? r[t][0] : (g == 1 ? r[t][1] : r[t][2]);
        }
        uint32_t *o = rows + (i * P + (unsigned long long)sub * (P / PS)) * (unsigned long long)W + w;
        gt_walk<S, K>(r, p, o, W);
    }
}

// One thread per combination: its 2 x 3^K counts, tables[i][class][x].
template <int K>
__global__ void __launch_bounds__(256) ct_kernel(DsView d, const int32_t *__restrict__ combos, unsigned long long n,
                                                 uint32_t *__restrict__ tables, int *__restrict__ err) {
    for (unsigned long long i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (unsigned long long)gridDim.x * 256ull) {
        int c[K];
        bool bad = false;
        #pragma unroll
        for (int t = 0; t < K; ++t) {
            const int sn = combos[i * K + t];
            bad |= sn < 0 || sn >= d.M;
            c[t] = sn < 0 || sn >= d.M ? 0 : sn;
        }
        if (bad) {
            atomicOr(err, 1);
            continue;
        }
        (void)generic_num<K, true>(d, c, 0, tables + i * (2ull * pow3c(K)), 1);
    }
}

// N * MI of a table by Equation 1 from the exact n ln n table, as the scans
// score a combination, then MI = that / 2^shift / N; a table whose classes do
// not sum to the dataset's class sizes is rejected.  One lane per table, 64
// tables per wave: the wave stages kMiChunk cells of both classes of each of
// its tables into its LDS slot (each class's cells read as consecutive
// words), then every lane sums its own table's terms from there.  With LDT
// the n ln n table (n = 0 .. N) is staged at LDS address 0 first.
constexpr int kMiChunk = 16;
constexpr int kMiRow = 2 * kMiChunk + 1;  // words per table in a slot; the odd stride keeps lanes on distinct banks

template <bool LDT>
__global__ void __launch_bounds__(256) mi_kernel(DsView d, int P, long long score_const,
                                                 const uint32_t *__restrict__ tables, unsigned long long n,
                                                 double *__restrict__ mi, int *__restrict__ err) {
    // dynamic LDS: [LDT: 2 (N + 1) words of n ln n table][4 waves x 64 x kMiRow words of staged cells]
    extern __shared__ __attribute__((aligned(16))) unsigned char s_mi[];
    unsigned *s_t = (unsigned *)s_mi;
    const int tl_words = LDT ? (2 * (d.N + 1) + 3) & ~3 : 0;
    unsigned *slot = s_t + tl_words + (threadIdx.x >> 6) * (64 * kMiRow);
    bool at0 = false;  // the lookups address the staged table from LDS address 0
    if constexpr (LDT) {
        const unsigned *src = (const unsigned *)d.tlog;
        for (int x = threadIdx.x; x < 2 * (d.N + 1); x += blockDim.x) s_t[x] = src[x];
        __syncthreads();
        at0 = (unsigned)(uintptr_t)(lu32 *)s_t == 0u;
    }
    const int lane = threadIdx.x & 63;
    const unsigned long long groups = (n + 63) / 64;
    const unsigned long long n_waves = (unsigned long long)gridDim.x * 4;
    for (unsigned long long g = blockIdx.x * 4ull + (threadIdx.x >> 6); g < groups; g += n_waves) {
        const unsigned long long i0 = g * 64;
        const int nt = (int)min(64ull, n - i0);
        long long num = score_const;
        unsigned long long s0 = 0, s1 = 0;
        bool ok = true;
        for (int c0 = 0; c0 < P; c0 += kMiChunk) {
            const int cw = min(kMiChunk, P - c0), row = 2 * cw;
            for (int j = lane; j < nt * row; j += 64) {
                const int t = j / row, r = j - t * row, cl = r >= cw ? 1 : 0, x = r - cl * cw;
                slot[t * kMiRow + cl * kMiChunk + x] =
                    tables[(i0 + t) * 2ull * (unsigned)P + (unsigned)(cl * P + c0 + x)];
            }
            wave_sync();
            if (lane < nt) {
                for (int x = 0; x < cw; ++x) {
                    const unsigned n0 = slot[lane * kMiRow + x], n1 = slot[lane * kMiRow + kMiChunk + x];
                    const bool in = n0 <= (unsigned)d.ncls[0] && n1 <= (unsigned)d.ncls[1];
                    ok &= in;
                    s0 += n0;
                    s1 += n1;
                    num += in ? (LDT && at0 ? cell_term_lds(n0, n1) : cell_term_counted(d.tlog, n0, n1)) : 0;
                }
            }
            wave_sync();
        }
        if (lane < nt) {
            ok &= s0 == (unsigned long long)d.ncls[0] && s1 == (unsigned long long)d.ncls[1];
            mi[i0 + lane] = ok ? ldexp((double)num, -d.shift) / (double)d.N : __builtin_nan("");
            if (!ok) atomicOr(err, 1);
        }
    }
}

size_t mi_lds_bytes(int N, bool ldt) {
    return (ldt ? (size_t)4 * ((2 * (N + 1) + 3) & ~3) : 0) + (size_t)4 * 4 * 64 * kMiRow;
}

template <int K>
static hipError_t launch_function_k(int fn, hipStream_t st, const DsView &d, const int32_t *combos,
                                    unsigned long long n, void *out, int *err, int grid) {
    if (fn == 0) {
        hipLaunchKernelGGL(gt_kernel<K>, dim3(grid), dim3(256), 0, st, d, combos, n, (uint32_t *)out, err);
    } else {
        if constexpr (K < 2) return hipErrorInvalidValue;  // tables start at order 2
        else hipLaunchKernelGGL(ct_kernel<K>, dim3(grid), dim3(256), 0, st, d, combos, n, (uint32_t *)out, err);
    }
    return hipGetLastError();
}

hipError_t launch_function(int fn, int order, hipStream_t st, const DsView &d, const int32_t *combos,
                           const uint32_t *tables, unsigned long long n, void *out, int *err, int grid,
                           long long score_const) {
    if (fn == 2) {
        // the exact table in LDS when it fits beside two workgroups per CU
        if ((size_t)8 * (d.N + 1) <= 64 * 1024)
            hipLaunchKernelGGL(mi_kernel<true>, dim3(grid), dim3(256), mi_lds_bytes(d.N, true), st, d, pow3i(order),
                               score_const, tables, n, (double *)out, err);
        else
            hipLaunchKernelGGL(mi_kernel<false>, dim3(grid), dim3(256), mi_lds_bytes(d.N, false), st, d,
                               pow3i(order), score_const, tables, n, (double *)out, err);
        return hipGetLastError();
    }
    switch (order) {
    case 1: return launch_function_k<1>(fn, st, d, combos, n, out, err, grid);
    case 2: return launch_function_k<2>(fn, st, d, combos, n, out, err, grid);
    case 3: return launch_function_k<3>(fn, st, d, combos, n, out, err, grid);
    case 4: return launch_function_k<4>(fn, st, d, combos, n, out, err, grid);
    case 5: return launch_function_k<5>(fn, st, d, combos, n, out, err, grid);
    case 6: return launch_function_k<6>(fn, st, d, combos, n, out, err, grid);
    case 7: return launch_function_k<7>(fn, st, d, combos, n, out, err, grid);
    case 8: return launch_function_k<8>(fn, st, d, combos, n, out, err, grid);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Packing (Section 2.1): one thread per (SNP, 128-individual group of a
// class).  idx lists the input position of each class's individuals (cases
// first).  Genotypes outside {0,1,2} raise *err.
// ---------------------------------------------------------------------------
__global__ void pack_kernel(const uint8_t *__restrict__ geno, long long ld, const int32_t *__restrict__ idx, DsView d,
                            v4u *__restrict__ masks, int *__restrict__ err) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int G4 = d.w4[0] + d.w4[1];
    if (tid >= (long long)G4 * d.Mp) return;
    const int s = (int)(tid % d.Mp);
    const int g4 = (int)(tid / d.Mp);
    const int cl = g4 < d.w4[0] ? 0 : 1;
    const int w4 = g4 - d.wbase[cl];
    const int32_t *cidx = idx + (cl == 0 ? 0 : d.ncls[0]);
    v4u r0 = {0u, 0u, 0u, 0u}, r1 = {0u, 0u, 0u, 0u};
    int bad = 0;
    if (s < d.M) {
        const uint8_t *row = geno + (long long)s * ld;
        #pragma unroll
        for (int q = 0; q < 4; ++q) {
            unsigned b0 = 0, b1 = 0;
            for (int b = 0; b < 32; ++b) {
                const int pos = 32 * (4 * w4 + q) + b;
                if (pos < d.ncls[cl]) {
                    const unsigned si = (unsigned)cidx[pos];
                    if (si >= (unsigned)d.N) {
                        bad |= 8;
                        continue;
                    }
                    const unsigned g = row[si];
                    b0 |= (g == 0u ? 1u : 0u) << b;
                    b1 |= (g == 1u ? 1u : 0u) << b;
                    bad |= g > 2u ? 1 : 0;
                }
            }
            r0[q] = b0;
            r1[q] = b1;
        }
    }
    masks[((long long)g4 * 2 + 0) * d.Mp + s] = r0;
    masks[((long long)g4 * 2 + 1) * d.Mp + s] = r1;
    if (bad) atomicOr(err, bad);
}

__global__ void singles_kernel(DsView d, uint32_t *__restrict__ single) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= d.Mp * 2) return;
    const int s = tid >> 1, cl = tid & 1;
    gv4u *gm = (gv4u *)d.masks;
    unsigned n0 = 0, n1 = 0;
    long long off = (long long)d.wbase[cl] * 2 * d.Mp;
    for (int w = 0; w < d.w4[cl]; ++w, off += 2 * d.Mp) {
        const v4u r0 = gm[off + s], r1 = gm[off + d.Mp + s];
        #pragma unroll
        for (int q = 0; q < 4; ++q) {
            n0 += __builtin_popcount(r0[q]);
            n1 += __builtin_popcount(r1[q]);
        }
    }
    single[(s * 2 + cl) * 2 + 0] = n0;
    single[(s * 2 + cl) * 2 + 1] = n1;
}

// Matrix-core operand copies of the genotype-0/1 rows: one thread per (SNP,
// genotype, 64-individual step, half); each 32-individual mask word becomes
// 32 4-bit floats, low nibble first: 0x2 = 1.0 (qa) or 0x6 = 4.0 (qb) for a
// set bit.
__global__ void qpack_kernel(DsView d, v4u *__restrict__ qa, v4u *__restrict__ qb) {
    const long long KS = d.ks[0] + d.ks[1];
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (long long)d.Mp * 2 * KS * 2) return;
    const int s = (int)(tid % d.Mp);
    long long rest = tid / d.Mp;
    const int g = (int)(rest & 1);
    rest >>= 1;
    const int h = (int)(rest & 1);
    const long long step = rest >> 1;
    const int c = step < d.ks[0] ? 0 : 1;
    const int widx = 2 * (int)(step - (c == 0 ? 0 : d.ks[0])) + h;  // 32-bit word within the class
    unsigned word = 0;
    if ((widx >> 2) < d.w4[c]) {
        gv4u *gm = (gv4u *)d.masks;
        word = gm[((long long)(d.wbase[c] + (widx >> 2)) * 2 + g) * d.Mp + s][widx & 3];
    }
    // qa: 1.0 = 0x2 per set bit; qb: 4.0 = 0x6 (counts come out as 4 n)
    v4u out;
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
        unsigned x = 0;
        #pragma unroll
        for (int t = 0; t < 4; ++t) {
            const unsigned b = (word >> (8 * k + 2 * t)) & 3u;
            x |= (((b & 1u) << 1) | ((b >> 1) << 5)) << (8 * t);
        }
        out[k] = x;
    }
    qa[((long long)(s >> 4) * KS + step) * 64 + 32 * h + 2 * (s & 15) + g] = out;
    qb[(((long long)(s >> 5) * 2 + g) * KS + step) * 64 + 32 * h + (s & 31)] = out | (out << 1);
}

// Integer operand copies: one thread per (SNP, genotype, 32-individual step,
// half); each 16-individual half word becomes 16 bytes, 1 (qa8) or 4 (qb8)
// per set bit.
__global__ void qpack8_kernel(DsView d, v4u *__restrict__ qa8, v4u *__restrict__ qb8) {
    const long long KS = d.ks8[0] + d.ks8[1];
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (long long)d.Mp * 2 * KS * 2) return;
    const int s = (int)(tid % d.Mp);
    long long rest = tid / d.Mp;
    const int g = (int)(rest & 1);
    rest >>= 1;
    const int h = (int)(rest & 1);
    const long long step = rest >> 1;
    const int c = step < d.ks8[0] ? 0 : 1;
    const int widx = (int)(step - (c == 0 ? 0 : d.ks8[0]));  // 32-bit word within the class
    unsigned word = 0;
    if ((widx >> 2) < d.w4[c]) {
        gv4u *gm = (gv4u *)d.masks;
        word = gm[((long long)(d.wbase[c] + (widx >> 2)) * 2 + g) * d.Mp + s][widx & 3];
    }
    const unsigned half = word >> (16 * h);
    v4u out;
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
        unsigned x = 0;
        #pragma unroll
        for (int t = 0; t < 4; ++t) x |= ((half >> (4 * k + t)) & 1u) << (8 * t);
        out[k] = x;
    }
    qa8[((long long)(s >> 4) * KS + step) * 64 + 32 * h + 2 * (s & 15) + g] = out;
    qb8[(((long long)(s >> 5) * 2 + g) * KS + step) * 64 + 32 * h + (s & 31)] = out << 2;  // 4 per set bit
}

// Class index map: idx[0 .. n_case) = input positions of the cases in input
// order, idx[n_case .. N) = those of the controls.  One 1024-thread
// workgroup, the first kernel of a packing: it clears the dataset's error
// word, then a phenotype outside {0,1} raises bit 2 and a number of cases
// other than n_case bit 4 (some index then falls outside its class).
__global__ void __launch_bounds__(1024) classidx_kernel(const uint8_t *__restrict__ pheno, int N, int n_case,
                                                        int32_t *__restrict__ idx, int *__restrict__ err) {
    __shared__ int s_scan[1024];
    __shared__ int s_cases;
    const int tid = threadIdx.x;
    if (tid == 0) {
        s_cases = 0;
        *err = 0;
    }
    __syncthreads();
    for (int base = 0; base < N; base += 1024) {
        const int s = base + tid;
        int f = 0;
        if (s < N) {
            const unsigned v = pheno[s];
            f = v == 1u ? 1 : 0;
            if (v > 1u) atomicOr(err, 2);
        }
        s_scan[tid] = f;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int v = tid >= off ? s_scan[tid - off] : 0;
            __syncthreads();
            s_scan[tid] += v;
            __syncthreads();
        }
        const int before = s_scan[tid] - f;  // cases before s within this chunk
        const int bc = s_cases;
        if (s < N) {
            if (f) {
                if (bc + before < n_case) idx[bc + before] = s;
                else atomicOr(err, 4);
            } else {
                const int pos = n_case + (base - bc) + (tid - before);
                if (pos < N) idx[pos] = s;
                else atomicOr(err, 4);
            }
        }
        __syncthreads();
        if (tid == 1023) s_cases = bc + s_scan[1023];
        __syncthreads();
    }
}

// After a merge: the best K (results) become the first entries of each
// task's candidate buffer, so later launches of the same task (serving
// rounds) add to a compact list.
__global__ void reseed_kernel(const Task *__restrict__ tasks, const Cand *__restrict__ results) {
    const Task &t = tasks[blockIdx.x];
    const Cand *res = results + (long long)blockIdx.x * kMaxTopK;
    int n = 0;
    for (int r = 0; r < t.top_k; ++r) n += res[r].key != ~0ull ? 1 : 0;
    for (int r = threadIdx.x; r < n; r += blockDim.x) t.cand[r] = res[r];
    if (threadIdx.x == 0) *t.cand_count = (unsigned)n;
}

// Work-item descriptor table of one shape (kinds and layouts in
// epi_internal.hpp), written by one workgroup: the groups go 1024 at a time,
// a scan of their sizes gives each its offset, and each thread writes the
// items of its group.  out holds exactly the sum of the group sizes, which
// the host counts with the same functions.
__global__ void __launch_bounds__(1024) items_kernel(int kind, int M, int np, unsigned long long *__restrict__ out) {
    __shared__ unsigned long long s_scan[1024];
    __shared__ unsigned long long s_base;
    const long long G = item_groups(kind, M, np);
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    for (long long g0 = 0; g0 < G; g0 += 1024) {
        const long long g = g0 + threadIdx.x;
        ItemGroup gr{0, 1, 0, 0};
        if (g < G) gr = item_group(kind, M, np, g);
        s_scan[threadIdx.x] = gr.count;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const unsigned long long v = (int)threadIdx.x >= off ? s_scan[threadIdx.x - off] : 0ull;
            __syncthreads();
            s_scan[threadIdx.x] += v;
            __syncthreads();
        }
        const unsigned long long start = s_base + s_scan[threadIdx.x] - gr.count;
        for (unsigned long long t = 0; t < gr.count; ++t) out[start + t] = item_at(gr, t);
        __syncthreads();
        if (threadIdx.x == 1023) s_base += s_scan[1023];
        __syncthreads();
    }
}

// Bytes carried to device memory in a kernel's arguments (the task array of
// a launch sequence that may not copy from host memory).
struct StoreChunk {
    unsigned char b[kStoreChunkBytes];
};

__global__ void store_kernel(StoreChunk payload, int n, unsigned char *__restrict__ dst) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = payload.b[i];
}

// A result block (layout in epi_internal.hpp) copied to separate buffers of
// the caller: combinations, scores and (tables non-null) tables of the
// n_valid results; *n receives n_valid, or -1 when the dataset's last packing
// had invalid input.
__global__ void scatter_kernel(const char *__restrict__ block, int top_k, int order, int32_t *__restrict__ combos,
                               float *__restrict__ scores, uint32_t *__restrict__ tables, int32_t *__restrict__ n) {
    const int32_t *hdr = (const int32_t *)block;
    const long long nv = hdr[0];
    const long long nc = nv * order, ns = nv, nt = tables ? nv * 2 * pow3c(order) : 0;
    const int32_t *src_c = (const int32_t *)(block + 16);
    const float *src_s = (const float *)(block + 16 + (long long)top_k * order * 4);
    const uint32_t *src_t = (const uint32_t *)(block + 16 + (long long)top_k * order * 4 + (long long)top_k * 4);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nc + ns + nt;
         i += (long long)gridDim.x * blockDim.x) {
        if (i < nc) combos[i] = src_c[i];
        else if (i < nc + ns) scores[i - nc] = src_s[i - nc];
        else tables[i - nc - ns] = src_t[i - nc - ns];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *n = hdr[1] ? -1 : (int32_t)nv;
}

// Counters of a launch sequence: queues, candidate counts, thresholds.
__global__ void init_counters_kernel(unsigned long long *queues, int nq, unsigned *cand_counts,
                                     unsigned long long *thrs, int n_tasks, unsigned *hist) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < nq) queues[tid] = 0;
    if (tid < n_tasks) {
        cand_counts[tid] = 0;
        thrs[tid] = 0;  // bias(INT64_MIN)
    }
    if (hist && tid < (long long)n_tasks * kHistWords) hist[tid] = 0;
}

// ---------------------------------------------------------------------------
// Host-side launchers (called by the runtime).
// ---------------------------------------------------------------------------
static const ScanKernelEntry kScanKernels[] = {EPI_SCAN_KERNELS(false)};

ScanKernelFn find_scan_kernel_check(int np2, int np3, int gk);  // the EPI_SCAN_CHECK build of this file

size_t scan_lds_bytes(int tab_cap, int kmax, int stage_cap) {
    return (((size_t)tab_cap * 4 + 15) & ~(size_t)15) + (size_t)4 * kmax * sizeof(Cand) +
           (size_t)4 * stage_cap * sizeof(v4u) + 2 * sizeof(unsigned long long);
}

ScanKernelFn find_scan_kernel(int np2, int np3, int gk) {
    for (const auto &e : kScanKernels)
        if (e.np2 == np2 && e.np3 == np3 && e.gk == gk) return e.fn;
    return nullptr;
}

// grid = number of 4-wave workgroups; check: the checking instantiation
hipError_t launch_scan(int np2, int np3, int gk, int grid, hipStream_t st, const Task *tasks, int n_tasks,
                       unsigned long long total_items, unsigned long long *queue, const unsigned long long *binom,
                       int bstride, int tab_cap, int kmax, int stage_cap, bool check) {
    ScanKernelFn fn = check ? find_scan_kernel_check(np2, np3, gk) : find_scan_kernel(np2, np3, gk);
    if (!fn) return hipErrorInvalidValue;
    const size_t lds = scan_lds_bytes(tab_cap, kmax, stage_cap);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(4 * kWave), lds, st, tasks, n_tasks, total_items, queue, binom, bstride,
                       tab_cap, kmax, stage_cap);
    return hipGetLastError();
}

hipError_t launch_pilot(int np2, int np3, int gk, int grid, hipStream_t st, const Task *tasks, int n_tasks,
                        unsigned long long total, const unsigned long long *binom, int bstride, int tab_cap, int kmax,
                        int stage_cap) {
    void (*fn)(const Task *, int, unsigned long long, const unsigned long long *, int, int, int, int) =
        gk == 4               ? scan_pilot<0, 0, 4>
        : np3 == kNpMfma      ? scan_pilot<0, kNpMfma, 0>
        : np3 == kNpMfmaI8    ? scan_pilot<0, kNpMfmaI8, 0>
        : np3 == kNpMfma2     ? scan_pilot<0, kNpMfma2, 0>
        : np2 == kNpMfma      ? scan_pilot<kNpMfma, 0, 0>
        : np2 == 2            ? scan_pilot<2, 0, 0>
        : np2 == 4            ? scan_pilot<4, 0, 0>
        : np2 == 8            ? scan_pilot<8, 0, 0>
                              : nullptr;
    if (!fn) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(4 * kWave), scan_lds_bytes(tab_cap, kmax, stage_cap), st, tasks, n_tasks,
                       total, binom, bstride, tab_cap, kmax, stage_cap);
    return hipGetLastError();
}

hipError_t launch_merge(int n_tasks, hipStream_t st, const Task *tasks, Cand *parts, Cand *results) {
    hipLaunchKernelGGL(merge_part_kernel, dim3(kMergeParts, n_tasks), dim3(1024), 0, st, tasks, parts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(merge_final_kernel, dim3(n_tasks), dim3(1024), 0, st, tasks, (const Cand *)parts, kMergeParts,
                       results);
    return hipGetLastError();
}

hipError_t scan_attributes(int np2, int np3, int gk, int *vgprs, int *lds_bytes) {
    ScanKernelFn fn = find_scan_kernel(np2, np3, gk);
    if (!fn) return hipErrorInvalidValue;
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, (const void *)fn);
    if (e != hipSuccess) return e;
    *vgprs = a.numRegs;
    *lds_bytes = (int)a.sharedSizeBytes;
    return hipSuccess;
}

hipError_t launch_finalize(int n_tasks, int max_k, hipStream_t st, const Task *tasks, const Cand *results,
                           const ResultLayout *layout, char *out) {
    hipLaunchKernelGGL(finalize_kernel, dim3(max_k, n_tasks), dim3(kWave), 0, st, tasks, results, layout, out);
    return hipGetLastError();
}

hipError_t launch_init_counters(hipStream_t st, unsigned long long *queues, int nq, unsigned *cand_counts,
                                unsigned long long *thrs, int n_tasks, unsigned *hist) {
    long long n = nq > n_tasks ? nq : n_tasks;
    if (hist && (long long)n_tasks * kHistWords > n) n = (long long)n_tasks * kHistWords;
    hipLaunchKernelGGL(init_counters_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, queues, nq,
                       cand_counts, thrs, n_tasks, hist);
    return hipGetLastError();
}

hipError_t launch_items(hipStream_t st, int kind, int M, int np, unsigned long long *out) {
    hipLaunchKernelGGL(items_kernel, dim3(1), dim3(1024), 0, st, kind, M, np, out);
    return hipGetLastError();
}

hipError_t launch_store(hipStream_t st, const void *src, size_t bytes, void *dst) {
    for (size_t off = 0; off < bytes; off += kStoreChunkBytes) {
        StoreChunk c;
        const size_t n = bytes - off < (size_t)kStoreChunkBytes ? bytes - off : (size_t)kStoreChunkBytes;
        memcpy(c.b, (const char *)src + off, n);
        hipLaunchKernelGGL(store_kernel, dim3(1), dim3(256), 0, st, c, (int)n, (unsigned char *)dst + off);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_scatter(hipStream_t st, const char *block, int top_k, int order, int32_t *combos, float *scores,
                          uint32_t *tables, int32_t *n) {
    const long long items = (long long)top_k * (order + 1 + (tables ? 2 * pow3i(order) : 0));
    const int grid = (int)((items + 255) / 256 + 1 < 1024 ? (items + 255) / 256 + 1 : 1024);
    hipLaunchKernelGGL(scatter_kernel, dim3(grid), dim3(256), 0, st, block, top_k, order, combos, scores, tables, n);
    return hipGetLastError();
}

hipError_t launch_reseed(int n_tasks, hipStream_t st, const Task *tasks, const Cand *results) {
    hipLaunchKernelGGL(reseed_kernel, dim3(n_tasks), dim3(64), 0, st, tasks, results);
    return hipGetLastError();
}

hipError_t launch_pack(hipStream_t st, const uint8_t *geno, long long ld, const int32_t *idx, const DsView &d,
                       v4u *masks, int *err) {
    const long long n = (long long)(d.w4[0] + d.w4[1]) * d.Mp;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, geno, ld, idx, d, masks, err);
    return hipGetLastError();
}

hipError_t launch_classidx(hipStream_t st, const uint8_t *pheno, int N, int n_case, int32_t *idx, int *err) {
    hipLaunchKernelGGL(classidx_kernel, dim3(1), dim3(1024), 0, st, pheno, N, n_case, idx, err);
    return hipGetLastError();
}

hipError_t launch_qpack(hipStream_t st, const DsView &d, v4u *qa, v4u *qb) {
    const long long n = (long long)d.Mp * 2 * (d.ks[0] + d.ks[1]) * 2;
    hipLaunchKernelGGL(qpack_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, qa, qb);
    return hipGetLastError();
}

hipError_t launch_qpack8(hipStream_t st, const DsView &d, v4u *qa8, v4u *qb8) {
    const long long n = (long long)d.Mp * 2 * (d.ks8[0] + d.ks8[1]) * 2;
    hipLaunchKernelGGL(qpack8_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, qa8, qb8);
    return hipGetLastError();
}

hipError_t launch_singles(hipStream_t st, const DsView &d, uint32_t *single) {
    const int n = d.Mp * 2;
    hipLaunchKernelGGL(singles_kernel, dim3((n + 255) / 256), dim3(256), 0, st, d, single);
    return hipGetLastError();
}

#endif  // EPI_SCAN_CHECK

}  // namespace epi
