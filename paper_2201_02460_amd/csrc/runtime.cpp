// Host runtime of the epistasis scanner: contexts, a caching device
// allocator with a byte budget, resident datasets, scan plans (plain,
// back-to-back and persistent/graph-captured), the autotuner and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "../../include/epi.h"
#include "epi_internal.hpp"
#include "runtime_internal.hpp"

namespace epi {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string t_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

void clear_error() { t_err.clear(); }
const char *last_error() { return t_err.c_str(); }

#define HIPCHK(x)                                                                        \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) return fail(EPI_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// caching device allocator with a byte budget
// ---------------------------------------------------------------------------
static size_t round_size(size_t b) {
    if (b == 0) b = 1;
    if (b >= (1u << 20)) return (b + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1);
    size_t p = 256;
    while (p < b) p <<= 1;
    return p;
}

int DevAlloc::alloc(size_t bytes, void **out) {
    std::lock_guard<std::mutex> g(mu);
    const size_t sz = round_size(bytes);
    if (used + sz > budget) return fail(EPI_ENOMEM, "device budget exceeded: %zu used + %zu requested > %zu", used, sz, budget);
    auto it = free_.find(sz);
    void *p = nullptr;
    if (it != free_.end()) {
        p = it->second;
        free_.erase(it);
        cached -= sz;
    } else {
        hipError_t e = hipMalloc(&p, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trim_locked();
            e = hipMalloc(&p, sz);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return fail(EPI_ENOMEM, "hipMalloc(%zu) failed: %s", sz, hipGetErrorString(e));
            }
        }
    }
    live[p] = sz;
    used += sz;
    peak = std::max(peak, used);
    *out = p;
    return EPI_OK;
}

void DevAlloc::release(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu);
    auto it = live.find(p);
    if (it == live.end()) return;
    used -= it->second;
    cached += it->second;
    free_.emplace(it->second, p);
    live.erase(it);
}

void DevAlloc::trim_locked() {
    for (auto &kv : free_) (void)hipFree(kv.second);
    free_.clear();
    cached = 0;
}

void DevAlloc::trim() {
    std::lock_guard<std::mutex> g(mu);
    trim_locked();
}

void DevAlloc::destroy() {
    std::lock_guard<std::mutex> g(mu);
    trim_locked();
    for (auto &kv : live) (void)hipFree(kv.first);
    live.clear();
    used = 0;
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
uint64_t binom_u64(int64_t n, int64_t k) {
    if (k < 0 || n < 0 || k > n) return 0;
    if (k > n - k) k = n - k;
    unsigned __int128 r = 1;
    for (int64_t i = 0; i < k; ++i) {
        r = r * (unsigned __int128)(n - i) / (unsigned __int128)(i + 1);
        if (r > (unsigned __int128)UINT64_MAX) return UINT64_MAX;
    }
    return (uint64_t)r;
}

int key_bits_for(int order) { return 64 / order; }

// ---------------------------------------------------------------------------
// Scratch of the allocation-free scan (epi_scan_noalloc): a fixed array in
// every device's memory, held from the library's load until the process
// ends.  In host code `scratch` names a host-side stand-in, not the device
// array: its device address is taken once per device, at the first context
// created on that device, and only that address is used.  Every
// allocation-free scan on a device uses the whole array, so such calls must
// not overlap on one device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, char *> g_scratch_ptr;  // device -> address of its scratch array

// The device's scratch address (the device must be current).
static int scratch_of(int device, char **out) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it == g_scratch_ptr.end()) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(EPI_EDEVICE, "scratch array of device %d: %s", device, hipGetErrorString(e));
        it = g_scratch_ptr.emplace(device, (char *)ptr).first;
    }
    *out = it->second;
    return EPI_OK;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
Ctx *as_ctx(epi_ctx *c) { return reinterpret_cast<Ctx *>(c); }

int ctx_init(Ctx *c, int device, uint64_t budget) {
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(EPI_EINVAL, "device %d not in [0, %d)", device, n);
    c->device = device;
    HIPCHK(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    c->n_cu = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    c->arch = c->arch.substr(0, c->arch.find(':'));  // "gfx950:sramecc+:xnack-" -> "gfx950"
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    c->alloc.budget = budget ? budget : (uint64_t)(0.9 * (double)fr);
    HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    if (int rc = scratch_of(device, &c->scratch)) return rc;
    // binomial table for colex unranking: rows t = 0..kMaxBinomOrder, n = 0..kBinomN-1
    c->bstride = kBinomN;
    std::vector<unsigned long long> h((size_t)(kMaxBinomOrder + 1) * kBinomN);
    for (int t = 0; t <= kMaxBinomOrder; ++t)
        for (int n2 = 0; n2 < kBinomN; ++n2) h[(size_t)t * kBinomN + n2] = binom_u64(n2, t);
    int rc = c->alloc.alloc(h.size() * 8, (void **)&c->d_binom);
    if (rc) return rc;
    HIPCHK(hipMemcpy(c->d_binom, h.data(), h.size() * 8, hipMemcpyHostToDevice));
    const char *tc = getenv("EPI_TUNE_CACHE");
    if (tc) {
        c->tune_path = tc;
        load_tune_cache(c);
    }
    return EPI_OK;
}

// ---------------------------------------------------------------------------
// datasets
// ---------------------------------------------------------------------------
static int choose_shift(int N) {
    const double maxv = 2.0 * N * std::log(2.0 * std::max(N, 2)) + 1.0;
    int s = (int)std::floor(61.0 - std::log2(maxv));
    return std::min(40, std::max(8, s));
}

// Scale of the 32-bit screening table: a combination's screening sum is
// 2^tq times its score minus the class-split constant, which lies in
// [-N ln 2, 0] (Eq. 2: minus the entropy of the class within each cell,
// summed over the cells); 2^tq (N ln 2 + 1) <= 2^30 keeps it, with the
// rounding of the table values, inside int32, and the sum may wrap on the
// way there.  tq <= shift keeps the screening margin at one unit per value.
static int choose_tq(int N, int shift) {
    const double span = (double)N * std::log(2.0) + 1.0;
    const int q = (int)std::floor(30.0 - std::log2(span));
    return std::max(0, std::min(q, shift));
}

// round(n ln n * 2^shift) for n = 0 .. 2N (entries past N keep clamped
// lookups in bounds; valid tables never reach them).
static void build_tlog(int N, int shift, std::vector<long long> &out) {
    out.assign((size_t)2 * N + 1, 0);
    const long double sc = std::ldexp((long double)1.0, shift);
    for (int n = 2; n <= 2 * N; ++n) out[n] = llroundl((long double)n * logl((long double)n) * sc);
}

static void ds_free(Ctx *c, Dataset *d) {
    c->alloc.release(d->masks);
    c->alloc.release(d->single);
    c->alloc.release(d->tlog);
    c->alloc.release(d->itab);
    c->alloc.release(d->idx);
    c->alloc.release(d->err);
    c->alloc.release(d->qa);
    c->alloc.release(d->qb);
    c->alloc.release(d->qa8);
    c->alloc.release(d->qb8);
    d->masks = d->single = d->tlog = d->itab = d->idx = d->err = d->qa = d->qb = d->qa8 = d->qb8 = nullptr;
}

static int ds_layout(Dataset *d, int M, int N, int n_case) {
    d->M = M;
    d->N = N;
    d->n_case = n_case;
    d->n_ctrl = N - n_case;
    d->Mp = (M + 63) / 64 * 64;
    d->w4[0] = (d->n_case + 127) / 128;
    d->w4[1] = (d->n_ctrl + 127) / 128;
    const int q = 64 * kQStepMultiple;
    d->ks[0] = (d->n_case + q - 1) / q * kQStepMultiple;
    d->ks[1] = (d->n_ctrl + q - 1) / q * kQStepMultiple;
    const int q8 = 32 * kQStepMultiple;
    d->ks8[0] = (d->n_case + q8 - 1) / q8 * kQStepMultiple;
    d->ks8[1] = (d->n_ctrl + q8 - 1) / q8 * kQStepMultiple;
    d->shift = choose_shift(N);
    d->tq = choose_tq(N, d->shift);
    return EPI_OK;
}

static void ds_view(Dataset *d) {
    DsView &v = d->view;
    v.masks = (const v4u *)d->masks;
    v.single = (const uint32_t *)d->single;
    v.tlog = (const long long *)d->tlog;
    v.itab = (const uint32_t *)d->itab;
    v.tq = d->tq;
    v.M = d->M;
    v.Mp = d->Mp;
    v.N = d->N;
    v.shift = d->shift;
    v.ncls[0] = d->n_case;
    v.ncls[1] = d->n_ctrl;
    v.w4[0] = d->w4[0];
    v.w4[1] = d->w4[1];
    v.wbase[0] = 0;
    v.wbase[1] = d->w4[0];
    v.qa = (const v4u *)d->qa;
    v.qb = (const v4u *)d->qb;
    v.ks[0] = d->ks[0];
    v.ks[1] = d->ks[1];
    v.qa8 = (const v4u *)d->qa8;
    v.qb8 = (const v4u *)d->qb8;
    v.ks8[0] = d->ks8[0];
    v.ks8[1] = d->ks8[1];
    v.err = (const int *)d->err;
}

// Bytes of each integer operand copy.
static size_t qop8_bytes(const Dataset *d) { return (size_t)d->Mp * 2 * (d->ks8[0] + d->ks8[1]) * 32; }

// Bytes of each matrix-core operand copy (qa and qb hold the same rows).
static size_t qop_bytes(const Dataset *d) { return (size_t)d->Mp * 2 * (d->ks[0] + d->ks[1]) * 32; }

static int ds_alloc(Ctx *c, Dataset *d) {
    const size_t mask_bytes = (size_t)(d->w4[0] + d->w4[1]) * 2 * d->Mp * 16;
    int rc;
    if ((rc = c->alloc.alloc(std::max<size_t>(mask_bytes, 16), &d->masks))) return rc;
    if ((rc = c->alloc.alloc((size_t)d->Mp * 16, &d->single))) return rc;
    if ((rc = c->alloc.alloc(((size_t)2 * d->N + 1) * 8, &d->tlog))) return rc;
    if ((rc = c->alloc.alloc((size_t)d->N * 4, &d->idx))) return rc;
    if ((rc = c->alloc.alloc(((size_t)2 * d->N + 2) * 4, &d->itab))) return rc;
    if ((rc = c->alloc.alloc(256, &d->err))) return rc;
    d->bytes = mask_bytes + (size_t)d->Mp * 16 + ((size_t)2 * d->N + 1) * 8 + (size_t)d->N * 4;
    // float accumulation of 0/1 x 4 products is exact while 4 x a class count
    // stays below 2^24
    if (d->N < (1 << 22)) {
        if ((rc = c->alloc.alloc(qop_bytes(d), &d->qa))) return rc;
        if ((rc = c->alloc.alloc(qop_bytes(d), &d->qb))) return rc;
        d->bytes += 2 * qop_bytes(d);
    }
    ds_view(d);
    std::vector<long long> tl;
    build_tlog(d->N, d->shift, tl);
    HIPCHK(hipMemcpy(d->tlog, tl.data(), tl.size() * 8, hipMemcpyHostToDevice));
    // screening table: t(n) = round(n ln n 2^tq) mod 2^32, n = 0 .. N, then
    // the same values for n = N .. 0 (layout in epi_internal.hpp)
    std::vector<uint32_t> it((size_t)2 * d->N + 2, 0u);
    const long double tsc = std::ldexp((long double)1.0, d->tq);
    for (int n = 2; n <= d->N; ++n) {
        const uint32_t t = (uint32_t)(unsigned long long)llroundl((long double)n * logl((long double)n) * tsc);
        it[n] = t;
        it[(size_t)2 * d->N + 1 - n] = t;
    }
    HIPCHK(hipMemcpy(d->itab, it.data(), it.size() * 4, hipMemcpyHostToDevice));
    d->score_const = tl[d->N] - tl[d->n_case] - tl[d->n_ctrl];
    return EPI_OK;
}

// classidx + pack + singles, asynchronous on st
static int ds_pack(Dataset *d, const uint8_t *d_geno, int64_t ld, const uint8_t *d_pheno, hipStream_t st) {
    HIPCHK(launch_classidx(st, d_pheno, d->N, d->n_case, (int32_t *)d->idx, (int *)d->err));
    HIPCHK(launch_pack(st, d_geno, ld, (const int32_t *)d->idx, d->view, (v4u *)d->masks, (int *)d->err));
    HIPCHK(launch_singles(st, d->view, (uint32_t *)d->single));
    if (d->qa) HIPCHK(launch_qpack(st, d->view, (v4u *)d->qa, (v4u *)d->qb));
    if (d->qa8) HIPCHK(launch_qpack8(st, d->view, (v4u *)d->qa8, (v4u *)d->qb8));
    return EPI_OK;
}

// Integer operand copies of a dataset, built the first time the integer
// matrix-core kernel is selected for it (synchronous on the context stream).
static int ds_ensure_i8(Ctx *c, Dataset *d) {
    if (d->qa8) return EPI_OK;
    int rc;
    if ((rc = c->alloc.alloc(qop8_bytes(d), &d->qa8))) return rc;
    if ((rc = c->alloc.alloc(qop8_bytes(d), &d->qb8))) {
        c->alloc.release(d->qa8);
        d->qa8 = nullptr;
        return rc;
    }
    d->bytes += 2 * qop8_bytes(d);
    ds_view(d);
    HIPCHK(launch_qpack8(c->stream, d->view, (v4u *)d->qa8, (v4u *)d->qb8));
    HIPCHK(hipStreamSynchronize(c->stream));
    return EPI_OK;
}

static int load_common(Ctx *c, const uint8_t *d_geno, int64_t ld, const uint8_t *d_pheno,
                       const std::vector<uint8_t> &h_pheno, int32_t M, int32_t N, hipStream_t st,
                       int32_t *dataset_id) {
    int n_case = 0;
    for (int s = 0; s < N; ++s) {
        if (h_pheno[s] > 1) return fail(EPI_EINVAL, "phenotype of individual %d is %d (must be 0 or 1)", s, h_pheno[s]);
        n_case += h_pheno[s];
    }
    if (n_case == 0 || n_case == N) return fail(EPI_EINVAL, "need at least one case and one control (cases = %d of %d)", n_case, N);
    auto d = std::make_unique<Dataset>();
    ds_layout(d.get(), M, N, n_case);
    int rc = ds_alloc(c, d.get());
    if (rc) {
        ds_free(c, d.get());
        return rc;
    }
    rc = ds_pack(d.get(), d_geno, ld, d_pheno, st);  // the first kernel clears the error word
    int herr = 0;
    if (!rc) {
        hipError_t e = hipMemcpyAsync(&herr, d->err, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(EPI_EDEVICE, "dataset pack: %s", hipGetErrorString(e));
    }
    if (!rc && herr) rc = pack_error(herr);
    if (rc) {
        ds_free(c, d.get());
        return rc;
    }
    std::lock_guard<std::mutex> g(c->mu);
    d->id = c->next_id++;
    *dataset_id = d->id;
    c->datasets[d->id] = std::move(d);
    return EPI_OK;
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
int tuned_np_lookup(Ctx *c, int order, const Dataset *d) {
    const int bucket = size_bucket(d);
    std::lock_guard<std::mutex> g(c->tune_mu);
    auto it = c->tuned.find(TuneKey{order, bucket});
    return it != c->tuned.end() ? it->second : 0;
}

bool seg_pinned(Ctx *c, int order, const Dataset *d) {
    const int bucket = size_bucket(d);
    std::lock_guard<std::mutex> g(c->tune_mu);
    return c->seg_pins.count(TuneKey{order, bucket}) != 0;
}

static int tuned_np(Ctx *c, int order, const Dataset *d) {
    if (order == 3) return default_np3(c, d);
    const int t = tuned_np_lookup(c, order, d);
    if (t > 0 && (order != 2 || t != kNpMfma || d->qa)) return t;
    return order == 2 ? 4 : kGenRanksHost;
}

// Work items of the order-2 and order-3 kernels: kinds, groups and item
// layouts in epi_internal.hpp (item_group); the device writes the tables
// (items_kernel) and the host only counts their items.
static int item_kind(int variant, int np) {
    if (variant != kF3) return np == kNpMfma ? kItemsF2M : kItemsF2;
    if (np == kNpMfma2) return kItemsF3M2;
    return is_mfma_np(np) ? kItemsF3M : kItemsF3;
}

static unsigned long long item_count(int kind, int M, int np) {
    unsigned long long n = 0;
    const long long G = item_groups(kind, M, np);
    for (long long g = 0; g < G; ++g) n += item_group(kind, M, np, g).count;
    return n;
}

// Descriptor table of a shape, built once per context and cached.
int get_items(Ctx *c, int variant, int M, int np, const void **d, unsigned long long *n) {
    std::lock_guard<std::mutex> g(c->items_mu);
    const auto key = std::make_tuple(variant, M, np);
    auto it = c->item_tables.find(key);
    if (it == c->item_tables.end()) {
        const int kind = item_kind(variant, np);
        ItemTable t;
        t.n = item_count(kind, M, np);
        int rc = c->alloc.alloc(std::max<unsigned long long>(t.n, 1) * 8, &t.d);
        if (rc) return rc;
        if (t.n) {
            hipError_t e = launch_items(c->stream, kind, M, np, (unsigned long long *)t.d);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) {
                c->alloc.release(t.d);
                return fail(EPI_EDEVICE, "descriptor table: %s", hipGetErrorString(e));
            }
        }
        it = c->item_tables.emplace(key, t).first;
    }
    *d = it->second.d;
    *n = it->second.n;
    return EPI_OK;
}

// Device buffer of a plan: from the context's allocator, or (allocation-free
// plans) the next 256-byte-aligned piece of the scratch array.
static int plan_alloc(Ctx *c, Plan *p, size_t bytes, void **out) {
    if (!p->arena) return c->alloc.alloc(bytes, out);
    const size_t at = (p->arena_used + 255) & ~(size_t)255;
    if (at + bytes > p->arena_cap)
        return fail(EPI_EUNSUPPORTED, "the allocation-free scan needs more than its %zu-byte scratch array",
                    p->arena_cap);
    *out = p->arena + at;
    p->arena_used = at + bytes;
    return EPI_OK;
}

// Descriptor table of a shape for a plan: the context's cached table, else
// (allocation-free plans) one built into the plan's scratch and uploaded by
// its run, else a new cached table.
static int plan_items(Ctx *c, Plan *p, int variant, int M, int np, const void **d, unsigned long long *n) {
    if (p->arena) {
        std::lock_guard<std::mutex> g(c->items_mu);
        auto it = c->item_tables.find(std::make_tuple(variant, M, np));
        if (it != c->item_tables.end()) {
            *d = it->second.d;
            *n = it->second.n;
            return EPI_OK;
        }
    }
    if (!p->arena) return get_items(c, variant, M, np, d, n);
    const int kind = item_kind(variant, np);
    const unsigned long long cnt = item_count(kind, M, np);
    void *dev = nullptr;
    if (int rc = plan_alloc(c, p, std::max<unsigned long long>(cnt, 1) * 8, &dev)) return rc;
    if (cnt) p->item_gens.push_back(Plan::ItemGen{kind, M, np, dev});
    *d = dev;
    *n = cnt;
    return EPI_OK;
}

// Pinned host buffer of at least `bytes` (power-of-two capacity) from the
// context's pool, or new.
static int host_buf_get(Ctx *c, size_t bytes, void **out, size_t *cap) {
    size_t n = 4096;
    while (n < bytes) n <<= 1;
    {
        std::lock_guard<std::mutex> g(c->pool_mu);
        auto it = c->host_pool.find(n);
        if (it != c->host_pool.end()) {
            *out = it->second;
            *cap = n;
            c->host_pool.erase(it);
            c->host_pool_bytes -= n;
            return EPI_OK;
        }
    }
    HIPCHK(hipHostMalloc(out, n, hipHostMallocDefault));
    *cap = n;
    return EPI_OK;
}

// Back to the pool (at most 256 MiB kept; the rest is freed).
static void host_buf_put(Ctx *c, void *p, size_t cap) {
    if (!p) return;
    {
        std::lock_guard<std::mutex> g(c->pool_mu);
        if (c->host_pool_bytes + cap <= (256ull << 20)) {
            c->host_pool.emplace(cap, p);
            c->host_pool_bytes += cap;
            return;
        }
    }
    (void)hipHostFree(p);
}

static int event_get(Ctx *c, hipEvent_t *e) {
    {
        std::lock_guard<std::mutex> g(c->pool_mu);
        if (!c->event_pool.empty()) {
            *e = c->event_pool.back();
            c->event_pool.pop_back();
            return EPI_OK;
        }
    }
    HIPCHK(hipEventCreate(e));
    return EPI_OK;
}

static void event_put(Ctx *c, hipEvent_t e) {
    if (!e) return;
    std::lock_guard<std::mutex> g(c->pool_mu);
    c->event_pool.push_back(e);
}

static void pools_free(Ctx *c) {
    std::lock_guard<std::mutex> g(c->pool_mu);
    for (auto &kv : c->host_pool) (void)hipHostFree(kv.second);
    c->host_pool.clear();
    c->host_pool_bytes = 0;
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    c->event_pool.clear();
}

void plan_free(Ctx *c, Plan *p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    for (auto &s : p->scans) {
        c->alloc.release(s.pairs);
        c->alloc.release(s.triples);
        c->alloc.release(s.seg);
        c->alloc.release(s.cand);
    }
    c->alloc.release(p->d_parts);
    c->alloc.release(p->d_tasks);
    c->alloc.release(p->d_counters);
    c->alloc.release(p->d_results);
    c->alloc.release(p->d_layout);
    c->alloc.release(p->d_out);
    host_buf_put(c, p->h_out, p->h_out_cap);
    if (!p->arena) host_buf_put(c, p->h_stage, p->h_stage_cap);
    p->h_out = p->h_stage = nullptr;
    for (auto &e : p->ev) event_put(c, e);
    for (auto &e : p->ev) e = nullptr;
}

int check_desc(Ctx *c, const epi_scan_desc &d, Dataset **out) {
    auto it = c->datasets.find(d.dataset_id);
    if (it == c->datasets.end()) return fail(EPI_ENOTFOUND, "unknown dataset %d", d.dataset_id);
    Dataset *ds = it->second.get();
    if (d.reserved != 0) return fail(EPI_EINVAL, "reserved field must be 0");
    if (d.order < EPI_MIN_ORDER) return fail(EPI_EINVAL, "order %d < %d", d.order, EPI_MIN_ORDER);
    if (d.order > ds->M) return fail(EPI_EINVAL, "order %d > M = %d", d.order, ds->M);
    if (d.order > EPI_MAX_ORDER) return fail(EPI_EUNSUPPORTED, "order %d > %d", d.order, EPI_MAX_ORDER);
    if (d.top_k < 1) return fail(EPI_EINVAL, "top_k %d < 1", d.top_k);
    if (d.top_k > EPI_MAX_TOP_K) return fail(EPI_EUNSUPPORTED, "top_k %d > %d", d.top_k, EPI_MAX_TOP_K);
    const int bits = key_bits_for(d.order);
    if (bits < 32 && ds->M > (1 << bits))
        return fail(EPI_EUNSUPPORTED, "M = %d exceeds 2^%d for order %d", ds->M, bits, d.order);
    if ((long long)ds->M >= kBinomN && d.order >= 4)
        return fail(EPI_EUNSUPPORTED, "M = %d too large for the order-%d kernel", ds->M, d.order);
    *out = ds;
    return EPI_OK;
}

// Kernel instantiation for a group of tasks in one persistent launch.
void pick_group_kernel(const std::vector<int> &orders, int np_hint, int *np2, int *np3, int *gk) {
    bool has2 = false, has3 = false;
    int gen = 0;
    for (int o : orders) {
        if (o == 2) has2 = true;
        else if (o == 3) has3 = true;
        else gen = o;
    }
    *np2 = 0;
    *np3 = 0;
    *gk = 0;
    if (gen) {  // a generic order runs in a group of its own
        *gk = gen;
        return;
    }
    const int h = np_hint <= 2 ? 2 : (np_hint <= 4 ? 4 : 8);
    if (has2) *np2 = np_hint == kNpMfma ? kNpMfma : h;  // order 2: a popcount block or the matrix cores
    if (has3) *np3 = has2 ? h : np_hint;
}

// Launch-group key of a scan: one group per kernel instantiation (orders 2
// and 3 are split by prefix block).
int group_of_order(int order, int np) {
    if (order == 2) return 20 + np;
    if (order == 3) return 30 + np;
    return order;
}

// Prefix block of an order-3 scan: the autotuned value for the dataset's
// size bucket if there is one, else the matrix-core kernel when the dataset
// has its operand copies, else 4.
int default_np3(Ctx *c, const Dataset *d) {
    const int t = tuned_np_lookup(c, 3, d);
    if (t > 0 && np3_usable(d, t)) return t;
    return d->qa ? kNpMfma : 4;
}

int pilot_items_for(int variant, int np, unsigned long long n_items, int top_k, int N, int tab_cap, int waves) {
    if (!((variant == kF3 && is_mfma_np(np)) || variant == kR4 || variant == kF2) || tab_cap < N + 1) return 0;
    const unsigned long long n = std::min<unsigned long long>((unsigned long long)waves, n_items / 32) & ~3ull;
    return n >= 2ull * (unsigned long long)std::max(top_k, 1) ? (int)n : 0;
}

int group_list_cap(int np2, int np3, int gk, int tab_cap, int top_k, int stage_cap) {
    const int big = list_cap(top_k);
    return wgs_per_cu(np2, np3, gk, tab_cap, big, stage_cap) >= wgs_per_cu(np2, np3, gk, tab_cap, top_k, stage_cap)
               ? big
               : top_k;
}

// Whether the dataset can run order-3 block np: the matrix-core blocks need
// their operand copies, and the two-middle-SNP one its class sizes to fit
// one float accumulator (q3_pack_fits).
bool np3_usable(const Dataset *d, int np) {
    if (np == kNpMfma) return d->qa != nullptr;
    if (np == kNpMfma2) return d->qa != nullptr && q3_pack_fits(d->n_case, d->n_ctrl);
    if (np == kNpMfmaI8) return d->qa8 != nullptr;
    return np == 1 || np == 2 || np == 4 || np == 8;
}

// Persistent grid, in 4-wave workgroups (one wave per SIMD each): as many as
// fit on the device by the kernel's VGPR count (512 registers per SIMD lane,
// at most 8 waves per SIMD) and LDS use (160 KiB per CU).
// EPI_WAVES_PER_SIMD overrides the register-based count.  Extra workgroups
// only queue: the work queue drains either way.
int wgs_per_cu(int np2, int np3, int gk, int tab_cap, int kmax, int stage_cap) {
    int vgprs = 128, lds_static = 0;
    if (scan_attributes(np2, np3, gk, &vgprs, &lds_static) != hipSuccess) {
        (void)hipGetLastError();
        vgprs = 128;
        lds_static = 0;
    }
    const int alloc = std::max(8, (vgprs + 7) / 8 * 8);
    int waves = std::min(8, 512 / alloc);
    if (const char *e = getenv("EPI_WAVES_PER_SIMD")) waves = std::max(1, std::min(16, atoi(e)));
    const size_t lds = scan_lds_bytes(tab_cap, kmax, stage_cap) + (size_t)lds_static;
    const int by_lds = (int)std::max<size_t>(1, (160 * 1024) / std::max<size_t>(lds, 1));
    return std::max(1, std::min(waves, by_lds));
}

int grid_for(Ctx *c, int np2, int np3, int gk, unsigned long long items, int tab_cap, int kmax, int stage_cap) {
    long long g = (long long)wgs_per_cu(np2, np3, gk, tab_cap, kmax, stage_cap) * c->n_cu;
    const long long need = (long long)((items + 3) / 4);
    if (g > need) g = std::max(1LL, need);
    return (int)g;
}

// Per-wave LDS slot (uint4 entries) for the staged prefix rows: 2 rows per
// prefix SNP (order 2: NP SNPs, order 3: NP + 1) times the words of one chunk
// (at most 16 groups of 4 words, 2048 individuals of a class, which keeps
// three 4-wave workgroups per CU next to an 8001-entry screening table).
int stage_cap_for(int np2, int np3, int w4_max) {
    if (np2 == kNpMfma) return 0;  // order 2 on the matrix cores stages nothing
    if (np3 == kNpMfma2) return 8 * kQStageSteps;  // two middle SNPs' mask rows: 4 entries per step each
    if (is_mfma_np(np3)) return 4 * kQStageSteps;  // j-mask rows: 4 entries per step
    const int rows = std::max(np2 > 0 ? 2 * np2 : 0, np3 > 0 ? 2 * (np3 + 1) : 0);
    if (rows == 0) return 0;
    return rows * std::max(1, std::min(w4_max, 16));
}

// Cell form of the pair sub-table a scan's pair pass writes (the consumers'
// signed cell form, layout in epi_internal.hpp).
void set_pair_form(Task &t, const Dataset *d, int order, int variant, int np) {
    const bool q3 = order == 3 && is_mfma_np(np);
    const bool r4 = variant == kR4;
    t.cell_shift = q3 ? kQScaleShift : 0;
    t.cell_bias = q3 ? q3_bias(d->N) : 0u;
    t.cell_neg = q3 ? 1 : 0;
    t.pair_colex = r4 ? 1 : 0;  // colex order, both classes of a cell in one word
}

// Bytes of a scan's pair sub-table (order 4 by reduced cells: 16 per pair,
// both classes of a cell in one word; else 32) and triplet sub-table (32 per
// triplet, both classes in one word).
uint64_t pair_table_bytes(int variant, int M) { return binom_u64(M, 2) * (variant == kR4 ? 16 : 32); }
uint64_t triple_table_bytes(int M) { return binom_u64(M, 3) * 32; }

// Screening-table entries a scan takes in LDS: the first half (N + 1) when
// it fits in kTabMax entries, else none (the exact score path for every
// combination); with `both`, the kernels in the signed cell form (matrix-core
// order 3, order 4 by reduced cells) take the mirrored half too (2N + 2 in
// all) when that fits.
int tab_entries_for(const Dataset *d, int variant, int np, bool both) {
    if (variant == kGeneric || variant == kSeg)  // exact int64 table, n = 0 .. N
        return 2 * (d->N + 1) <= Plan::kTabMax ? 2 * (d->N + 1) : 0;
    if (variant != kF2 && variant != kF3 && variant != kR4) return 0;
    const bool sgn = variant == kF3 && is_mfma_np(np);
    if (both && sgn && 2 * d->N + 2 <= Plan::kTabMax) return 2 * d->N + 2;
    return d->N + 1 <= Plan::kTabMax ? d->N + 1 : 0;
}

// A group's LDS table capacity from the largest tables of its scans with
// (cap_both) and without (cap_first) mirrored halves: the former only if it
// keeps as many workgroups per CU.  A workgroup reloads the table when a
// chunk of work starts another dataset, and takes the mirrored half for the
// chunks that use it when it fits the capacity.
// Whether a scan's screening table (its first half) costs its kernel
// workgroups per CU even with the smallest best-K list a launch group may
// give it (K entries): such scans go to launch groups of their own, so that
// they do not lower the occupancy of the others.
bool table_lowers_occupancy(const Dataset *d, int variant, int np, int order, int top_k) {
    const int np2 = order == 2 ? np : 0, np3 = order == 3 ? np : 0, gk = order >= 4 ? order : 0;
    const int stage = stage_cap_for(np2, np3, std::max(d->w4[0], d->w4[1]));
    const int ent = tab_entries_for(d, variant, np, false);
    return ent > 0 && wgs_per_cu(np2, np3, gk, ent, top_k, stage) < wgs_per_cu(np2, np3, gk, 0, top_k, stage);
}

int group_tab_cap(int np2, int np3, int gk, int cap_both, int cap_first, int kmax, int stage_cap) {
    if (cap_both <= cap_first) return cap_first;
    const int w_both = wgs_per_cu(np2, np3, gk, cap_both, kmax, stage_cap);
    const int w_first = wgs_per_cu(np2, np3, gk, cap_first, kmax, stage_cap);
    return w_both >= w_first ? cap_both : cap_first;
}

static void pick_tab_cap(const Plan *p, LaunchGroup &g) {
    int cap_both = 0, cap_first = 0;
    g.kmax = 1;
    g.stage_cap = stage_cap_for(g.np2, g.np3, 0);
    for (int i : g.scans) {
        const PlanScan &s = p->scans[i];
        g.kmax = std::max(g.kmax, s.desc.top_k);
        g.stage_cap = std::max(g.stage_cap, stage_cap_for(g.np2, g.np3, std::max(s.ds->w4[0], s.ds->w4[1])));
        cap_both = std::max(cap_both, tab_entries_for(s.ds, s.variant, s.np, true));
        cap_first = std::max(cap_first, tab_entries_for(s.ds, s.variant, s.np, false));
    }
    g.tab_cap = group_tab_cap(g.np2, g.np3, g.gk, cap_both, cap_first, g.kmax, g.stage_cap);
    g.kmax = group_list_cap(g.np2, g.np3, g.gk, g.tab_cap, g.kmax, g.stage_cap);
}

// Order 4 by reduced cells needs the dataset's matrix-core operands (for the
// triplet sub-table pass) and a triplet sub-table of C(M,3) x 64 bytes; larger
// ones take the per-combination kernel.
static constexpr unsigned long long kMaxTripleBytes = 8ull << 30;
// (its cells hold 4 n of each class in 16 bits: classes of at most 16383)
bool r4_fits(const Dataset *d) {
    return d->qa && triple_table_bytes(d->M) <= kMaxTripleBytes && d->n_case <= 16383 && d->n_ctrl <= 16383;
}
// Order 4 runs by reduced cells when they fit, unless the all-cell kernel is
// pinned for the dataset's size bucket.
bool use_r4(Ctx *c, const Dataset *d) { return r4_fits(d) && tuned_np_lookup(c, 4, d) != EPI_BLOCK_ALL_CELLS; }
static bool needs_pairs(const PlanScan &s) {
    return s.variant != kSeg && (s.desc.order == 3 || s.variant == kR4);
}

int plan_build(Ctx *c, const epi_scan_desc *descs, int n, bool persistent, bool graph, Plan **out,
               int force_np, bool check, const PlanArena *arena) {
    if (n < 1) return fail(EPI_EINVAL, "empty scan list");
    std::vector<Dataset *> dss(n);
    for (int i = 0; i < n; ++i) {
        int rc = check_desc(c, descs[i], &dss[i]);
        if (rc) return rc;
    }
    auto p = std::make_unique<Plan>();
    p->persistent = persistent;
    p->use_graph = graph;
    p->check = check;
    if (arena) {
        p->arena = arena->base;
        p->arena_cap = arena->cap;
    }
    p->scans.resize(n);
    int rc = EPI_OK;
    auto cleanup = [&](int code) {
        plan_free(c, p.get());
        return code;
    };
    // per-scan variant and prefix block
    for (int i = 0; i < n; ++i) {
        PlanScan &s = p->scans[i];
        s.desc = descs[i];
        s.ds = dss[i];
        s.n_combos = binom_u64(s.ds->M, s.desc.order);
        const int o = s.desc.order;
        if (force_np == EPI_BLOCK_SEGMENTED || (force_np <= 0 && !arena && seg_pinned(c, o, s.ds))) {
            s.variant = kSeg;
            s.np = kGenRanksHost;
            s.n_items = (s.n_combos + 64ull * kGenRanksHost - 1) / (64ull * kGenRanksHost);
        } else if (o == 2) {
            s.variant = kF2;
            s.np = force_np > 0 ? force_np : tuned_np(c, 2, s.ds);
        } else if (o == 3) {
            s.variant = kF3;
            s.np = force_np > 0 ? force_np : tuned_np(c, 3, s.ds);
        } else {
            // an allocation-free plan takes the reduced-cell order-4 kernel
            // only when its two sub-tables fit in half the scratch array
            const bool r4_room =
                !arena || triple_table_bytes(s.ds->M) + pair_table_bytes(kR4, s.ds->M) <= arena->cap / 2;
            bool r4 = o == 4 && r4_fits(s.ds) && r4_room;
            if (force_np == EPI_BLOCK_ALL_CELLS) r4 = false;
            else if (force_np != kForceReducedCells) r4 = r4 && use_r4(c, s.ds);
            s.variant = r4 ? kR4 : kGeneric;
            s.np = kGenRanksHost;
            s.n_items = (s.n_combos + 64ull * kGenRanksHost - 1) / (64ull * kGenRanksHost);
        }
    }
    // Scans of several orders over one dataset count the pairs once: an
    // order-2 scan is scored by the pair sub-table pass of a higher-order scan
    // of the same dataset in this plan (kF2Fold) and has no launch of its own.
    std::vector<int> fold_of(n, -1);  // scan j's pair pass scores scan fold_of[j]
    if (persistent) {
        for (int i = 0; i < n; ++i) {
            PlanScan &s = p->scans[i];
            if (s.variant != kF2) continue;
            for (int j = 0; j < n; ++j) {
                if (j == i || fold_of[j] >= 0 || p->scans[j].ds != s.ds || !needs_pairs(p->scans[j])) continue;
                fold_of[j] = i;
                s.variant = kF2Fold;
                s.n_items = 0;
                break;
            }
        }
    }
    // launch groups
    if (persistent) {
        // one launch group per kernel instantiation: order 2, order 3 per
        // prefix block, each generic order; apart from those, the scans
        // whose screening table would cost their kernel workgroups per CU
        // (a group's LDS table takes its largest dataset)
        std::map<int, LaunchGroup> by_key;
        for (int i = 0; i < n; ++i) {
            const PlanScan &s = p->scans[i];
            if (s.variant == kF2Fold) continue;  // runs in the pair pass
            const bool seg = s.variant == kSeg;
            int key = seg ? 200 + s.desc.order : group_of_order(s.desc.order, s.np);
            if (!seg && table_lowers_occupancy(s.ds, s.variant, s.np, s.desc.order, s.desc.top_k)) key += 100;
            LaunchGroup &g = by_key[key];
            g.scans.push_back(i);
            std::vector<int> orders{s.desc.order};
            pick_group_kernel(orders, s.np, &g.np2, &g.np3, &g.gk);
            if (seg) {
                g.np2 = g.np3 = 0;
                g.gk = kSegGk + s.desc.order;
            }
        }
        for (auto &kv : by_key) p->groups.push_back(kv.second);
    } else {
        for (int i = 0; i < n; ++i) {
            LaunchGroup g;
            const PlanScan &s = p->scans[i];
            if (s.variant == kSeg) {
                g.np2 = 0;
                g.np3 = 0;
                g.gk = kSegGk + s.desc.order;
            } else if (s.desc.order == 2) {
                g.np2 = s.np;
                g.np3 = 0;
                g.gk = 0;
            } else if (s.desc.order == 3) {
                g.np2 = 0;
                g.np3 = s.np;
                g.gk = 0;
            } else {
                g.np2 = 0;
                g.np3 = 0;
                g.gk = s.desc.order;
            }
            g.scans.push_back(i);
            p->groups.push_back(g);
        }
    }
    // work-item descriptor tables and order-3 sub-table buffers
    for (auto &s : p->scans) {
        if (s.variant == kF2 || s.variant == kF3) {
            if ((rc = plan_items(c, p.get(), s.variant, s.ds->M, s.np, &s.items, &s.n_items))) return cleanup(rc);
        }
        if (needs_pairs(s)) {
            s.emit_np = 4;
            if ((rc = plan_items(c, p.get(), kF2, s.ds->M, s.emit_np, &s.emit_items_d, &s.emit_items)))
                return cleanup(rc);
            const size_t pb = (size_t)pair_table_bytes(s.variant, s.ds->M);
            if ((rc = plan_alloc(c, p.get(), std::max<size_t>(pb, 32), &s.pairs))) return cleanup(rc);
        }
        if (s.variant == kR4) {
            if ((rc = plan_items(c, p.get(), kF3, s.ds->M, kNpMfma, &s.t3_items_d, &s.t3_items))) return cleanup(rc);
            const size_t tb = (size_t)triple_table_bytes(s.ds->M);
            if ((rc = plan_alloc(c, p.get(), std::max<size_t>(tb, 64), &s.triples))) return cleanup(rc);
        }
    }
    // tasks: [main tasks in scan order][pair passes][triplet passes]
    const int nt = n;
    int n_emit = 0, n_t3 = 0;
    for (auto &s : p->scans) {
        n_emit += needs_pairs(s) ? 1 : 0;
        n_t3 += s.variant == kR4 ? 1 : 0;
    }
    p->n_emit = n_emit;
    p->n_t3 = n_t3;
    for (auto &g : p->groups) {
        unsigned long long tot = 0;
        for (int i : g.scans) tot += p->scans[i].n_items;
        g.total_items = tot;
        pick_tab_cap(p.get(), g);
        g.grid = grid_for(c, g.np2, g.np3, g.gk, tot, g.tab_cap, g.kmax, g.stage_cap);
    }
    // pair-pass launch shape (kernel <4,0,0>) and triplet-pass shape (<0,kNpMfma,0>)
    unsigned long long emit_total = 0, t3_total = 0;
    for (auto &s : p->scans) {
        emit_total += needs_pairs(s) ? s.emit_items : 0;
        t3_total += s.variant == kR4 ? s.t3_items : 0;
    }
    int emit_w4 = 1;
    for (auto &s : p->scans)
        if (needs_pairs(s)) emit_w4 = std::max(emit_w4, std::max(s.ds->w4[0], s.ds->w4[1]));
    p->emit_stage = stage_cap_for(4, 0, emit_w4);
    for (int j = 0; j < n; ++j)
        if (fold_of[j] >= 0) p->emit_kmax = std::max(p->emit_kmax, list_cap(p->scans[fold_of[j]].desc.top_k));
    p->emit_grid = grid_for(c, 4, 0, 0, std::max<unsigned long long>(emit_total, 1), 0, p->emit_kmax, p->emit_stage);
    p->t3_total = t3_total;
    p->t3_stage = stage_cap_for(0, kNpMfma, 0);
    p->t3_grid = grid_for(c, 0, kNpMfma, 0, std::max<unsigned long long>(t3_total, 1), 0, 1, p->t3_stage);
    // candidate buffers and result layout
    long long out_bytes = 0;
    for (int i = 0; i < n; ++i) {
        PlanScan &s = p->scans[i];
        int grid = s.variant == kF2Fold ? p->emit_grid : 0;
        for (auto &g : p->groups)
            for (int j : g.scans)
                if (j == i) grid = g.grid;
        // each wave of the launch flushes at most top_k entries per task
        s.cand_cap = (unsigned)std::min<unsigned long long>((unsigned long long)grid * 4 * s.desc.top_k + 64,
                                                            0xffffffffull);
        if ((rc = plan_alloc(c, p.get(), (size_t)s.cand_cap * sizeof(Cand), &s.cand))) return cleanup(rc);
        if (s.variant == kSeg) {
            // one block of 64 tables (2 x 3^k counts each) per wave slot of the launch
            const size_t sb = (size_t)grid * 4 * 64 * 2 * (size_t)pow3i(s.desc.order) * 4;
            if ((rc = plan_alloc(c, p.get(), sb, &s.seg))) return cleanup(rc);
        }
        s.lay.offset = out_bytes;
        s.lay.top_k = s.desc.top_k;
        s.lay.order = s.desc.order;
        out_bytes += result_block_bytes(s.desc.top_k, s.desc.order);
    }
    p->out_bytes = out_bytes;
    const int nq = (int)p->groups.size() + 2;  // pair pass, triplet pass, groups
    // checking plans: two digest words per scan right after the queues, so
    // the counter reset clears them with the queues
    const int ndig = check ? 2 * nt : 0;
    p->n_queues = nq + ndig;
    const size_t cnt_bytes =
        (size_t)(nq + ndig) * 8 + (size_t)nt * 8 + (size_t)nt * 4 + (size_t)nt * kHistWords * 4;
    if ((rc = plan_alloc(c, p.get(), cnt_bytes, &p->d_counters))) return cleanup(rc);
    p->d_queues = (unsigned long long *)p->d_counters;
    p->d_digest = check ? p->d_queues + nq : nullptr;
    p->d_thr = p->d_queues + nq + ndig;
    p->d_cand_count = (unsigned *)(p->d_thr + nt);
    p->d_hist = p->d_cand_count + nt;
    if ((rc = plan_alloc(c, p.get(), (size_t)nt * kMaxTopK * sizeof(Cand), &p->d_results))) return cleanup(rc);
    if ((rc = plan_alloc(c, p.get(), (size_t)nt * kMergeParts * kMaxTopK * sizeof(Cand), &p->d_parts)))
        return cleanup(rc);
    if ((rc = plan_alloc(c, p.get(), (size_t)nt * sizeof(ResultLayout), &p->d_layout))) return cleanup(rc);
    if ((rc = plan_alloc(c, p.get(), (size_t)std::max<long long>(out_bytes, 256), &p->d_out))) return cleanup(rc);
    // pinned results, then (checking plans) the digest words of every scan;
    // allocation-free plans scatter their results on the device instead
    if (!arena && (rc = host_buf_get(c, (size_t)std::max<long long>(out_bytes, 256) + (size_t)ndig * 8, &p->h_out,
                                     &p->h_out_cap)))
        return cleanup(rc);
    std::vector<ResultLayout> lay(nt);
    for (int i = 0; i < nt; ++i) lay[i] = p->scans[i].lay;
    // task array: [main tasks in scan order][pair passes][triplet passes]
    //             [per-group launch copies (persistent)]
    std::vector<Task> tasks(nt + n_emit + n_t3);
    for (int i = 0; i < nt; ++i) {
        PlanScan &s = p->scans[i];
        Task &t = tasks[i];
        memset(&t, 0, sizeof t);
        t.ds = s.ds->view;
        t.pairs = (uint32_t *)s.pairs;
        t.triples = (uint32_t *)s.triples;
        t.seg = (uint32_t *)s.seg;
        t.items = (const unsigned long long *)s.items;
        t.n_items = s.n_items;
        t.item_base = 0;
        t.n_combos = s.n_combos;
        t.score_const = s.ds->score_const;
        t.cand = (Cand *)s.cand;
        t.cand_count = p->d_cand_count + i;
        t.thr = p->d_thr + i;
        t.hist = p->d_hist + (size_t)i * kHistWords;
        t.cand_cap = s.cand_cap;
        t.variant = s.variant;
        t.order = s.desc.order;
        t.top_k = s.desc.top_k;
        t.np = s.np;
        t.n_blocks = 0;
        t.key_bits = key_bits_for(s.desc.order);
        t.digest = check ? p->d_digest + 2 * i : nullptr;
        // pilot pass: consecutive items from the middle of the task
        s.pilot_n = 0;
        s.pilot_first = 0;
        for (const LaunchGroup &g : p->groups)
            if (std::find(g.scans.begin(), g.scans.end(), i) != g.scans.end())
                s.pilot_n = pilot_items_for(s.variant, s.np, s.n_items, s.desc.top_k, s.ds->N, g.tab_cap, g.grid * 4);
        s.pilot_first = (s.n_items - (unsigned long long)s.pilot_n) / 2;
        t.pilot_first = s.pilot_first;
        t.pilot_n = s.pilot_n;
        t.pilot_base = 0;
    }
    {
        int e = nt;
        unsigned long long base = 0;
        for (int i = 0; i < nt; ++i) {
            PlanScan &s = p->scans[i];
            if (!needs_pairs(s)) continue;
            s.emit_task = e;
            Task &t = tasks[e++];
            t = tasks[i];
            t.variant = kF2Emit;
            t.digest = nullptr;
            t.pilot_first = 0;
            t.pilot_n = 0;
            t.pilot_base = 0;
            t.items = (const unsigned long long *)s.emit_items_d;
            t.n_items = s.emit_items;
            t.item_base = persistent ? base : 0;
            base += s.emit_items;
            t.np = s.emit_np;
            t.n_blocks = 0;
            t.order = 2;
            set_pair_form(t, s.ds, s.desc.order, s.variant, s.np);
            if (fold_of[i] >= 0) {
                // this pass also scores the order-2 scan: its best-K state
                const Task &o2 = tasks[fold_of[i]];
                t.variant = kF2Fold;
                t.cand = o2.cand;
                t.cand_count = o2.cand_count;
                t.thr = o2.thr;
                t.hist = o2.hist;
                t.cand_cap = o2.cand_cap;
                t.top_k = o2.top_k;
                t.key_bits = o2.key_bits;
                t.n_combos = o2.n_combos;
                t.score_const = o2.score_const;
                t.digest = o2.digest;
            }
        }
        base = 0;
        for (int i = 0; i < nt; ++i) {
            PlanScan &s = p->scans[i];
            if (s.variant != kR4) continue;
            s.t3_task = e;
            Task &t = tasks[e++];
            t = tasks[i];
            t.variant = kF3Emit;
            t.digest = nullptr;
            t.pilot_first = 0;
            t.pilot_n = 0;
            t.pilot_base = 0;
            t.items = (const unsigned long long *)s.t3_items_d;
            t.n_items = s.t3_items;
            t.item_base = persistent ? base : 0;
            base += s.t3_items;
            t.np = kNpMfma;
            t.order = 3;
        }
    }
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        LaunchGroup &g = p->groups[gi];
        if (!persistent) {
            g.task_off = g.scans.front();
            g.pilot_total = (unsigned long long)tasks[g.task_off].pilot_n;
            continue;
        }
        g.task_off = (int)tasks.size();
        unsigned long long base = 0, pbase = 0;
        for (int i : g.scans) {
            Task t = tasks[i];
            t.item_base = base;
            base += t.n_items;
            t.pilot_base = pbase;
            pbase += (unsigned long long)t.pilot_n;
            tasks.push_back(t);
        }
        g.pilot_total = pbase;
    }
    if ((rc = plan_alloc(c, p.get(), tasks.size() * sizeof(Task), &p->d_tasks))) return cleanup(rc);
    // layout and task arrays staged in pinned memory; every run uploads them
    // on its own stream ahead of its kernels (no synchronous copy here)
    p->stage_layout_bytes = ((size_t)nt * sizeof(ResultLayout) + 255) & ~(size_t)255;
    p->stage_tasks_bytes = tasks.size() * sizeof(Task);
    if (arena) {
        p->h_stage_mem.resize(p->stage_layout_bytes + p->stage_tasks_bytes);
        p->h_stage = p->h_stage_mem.data();
        p->h_stage_cap = 0;  // not from the pinned pool
    } else if ((rc = host_buf_get(c, p->stage_layout_bytes + p->stage_tasks_bytes, &p->h_stage, &p->h_stage_cap))) {
        return cleanup(rc);
    }
    memcpy(p->h_stage, lay.data(), (size_t)nt * sizeof(ResultLayout));
    memcpy((char *)p->h_stage + p->stage_layout_bytes, tasks.data(), p->stage_tasks_bytes);
    p->emit_total = emit_total;
    if (!arena)
        for (auto &ev : p->ev)
            if ((rc = event_get(c, &ev))) return cleanup(rc);
    *out = p.release();
    return EPI_OK;
}

// Enqueue the whole launch sequence of a plan on st.  With timing, events
// bracket the sub-table pass, the main kernel and the merge/finalize of a
// single-scan plan.
static int plan_enqueue(Ctx *c, Plan *p, hipStream_t st, bool timing, unsigned long long item_cap) {
    const Task *tasks = (const Task *)p->d_tasks;
    const int nt = (int)p->scans.size();
    for (auto &g : p->item_gens) HIPCHK(launch_items(st, g.kind, g.M, g.np, (unsigned long long *)g.dst));
    if (p->arena) {
        // no copy from host memory: the arrays travel in kernel arguments
        HIPCHK(launch_store(st, p->h_stage, (size_t)nt * sizeof(ResultLayout), p->d_layout));
        HIPCHK(launch_store(st, (const char *)p->h_stage + p->stage_layout_bytes, p->stage_tasks_bytes, p->d_tasks));
    } else {
        HIPCHK(hipMemcpyAsync(p->d_layout, p->h_stage, (size_t)nt * sizeof(ResultLayout), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(p->d_tasks, (const char *)p->h_stage + p->stage_layout_bytes, p->stage_tasks_bytes,
                              hipMemcpyHostToDevice, st));
    }
    HIPCHK(launch_init_counters(st, p->d_queues, p->n_queues, p->d_cand_count, p->d_thr, nt, p->d_hist));
    int q = 0;
    const bool single = nt == 1 && !p->persistent;
    if (timing && single) HIPCHK(hipEventRecord(p->ev[1], st));
    if (p->persistent) {
        if (p->n_emit > 0) {
            HIPCHK(launch_scan(4, 0, 0, p->emit_grid, st, tasks + nt, p->n_emit, p->emit_total, p->d_queues + q,
                               c->d_binom, c->bstride, 0, p->emit_kmax, p->emit_stage, p->check));
        }
        ++q;
        if (p->n_t3 > 0) {
            HIPCHK(launch_scan(0, kNpMfma, 0, p->t3_grid, st, tasks + nt + p->n_emit, p->n_t3, p->t3_total,
                               p->d_queues + q, c->d_binom, c->bstride, 0, 1, p->t3_stage));
        }
        ++q;
        if (timing && single) HIPCHK(hipEventRecord(p->ev[2], st));
        for (auto &g : p->groups) {
            if (g.pilot_total > 0 && item_cap == ~0ull)
                HIPCHK(launch_pilot(g.np2, g.np3, g.gk, (int)std::min<unsigned long long>(g.grid, g.pilot_total / 4), st,
                                    tasks + g.task_off, (int)g.scans.size(), g.pilot_total, c->d_binom, c->bstride,
                                    g.tab_cap, g.kmax, g.stage_cap));
            HIPCHK(launch_scan(g.np2, g.np3, g.gk, g.grid, st, tasks + g.task_off, (int)g.scans.size(),
                               std::min(g.total_items, item_cap), p->d_queues + q, c->d_binom, c->bstride,
                               g.tab_cap, g.kmax, g.stage_cap, p->check));
            ++q;
        }
        if (timing && single) HIPCHK(hipEventRecord(p->ev[3], st));
        HIPCHK(launch_merge(nt, st, tasks, (Cand *)p->d_parts, (Cand *)p->d_results));
        int maxk = 1;
        for (auto &s : p->scans) maxk = std::max(maxk, s.desc.top_k);
        HIPCHK(launch_finalize(nt, maxk, st, tasks, (const Cand *)p->d_results, (const ResultLayout *)p->d_layout,
                               (char *)p->d_out));
    } else {
        // back-to-back: per scan, [pair pass] main merge finalize
        for (int i = 0; i < nt; ++i) {
            PlanScan &s = p->scans[i];
            LaunchGroup &g = p->groups[i];
            if (needs_pairs(s)) {
                const int es = stage_cap_for(4, 0, std::max(s.ds->w4[0], s.ds->w4[1]));
                const int eg = grid_for(c, 4, 0, 0, s.emit_items, 0, 1, es);
                HIPCHK(launch_scan(4, 0, 0, eg, st, tasks + s.emit_task, 1, s.emit_items, p->d_queues + 0,
                                   c->d_binom, c->bstride, 0, 1, es));
                HIPCHK(launch_init_counters(st, p->d_queues, 1, nullptr, nullptr, 0, nullptr));
            }
            if (s.variant == kR4) {
                const int ts = stage_cap_for(0, kNpMfma, 0);
                const int tg = grid_for(c, 0, kNpMfma, 0, s.t3_items, 0, 1, ts);
                HIPCHK(launch_scan(0, kNpMfma, 0, tg, st, tasks + s.t3_task, 1, s.t3_items, p->d_queues + 0,
                                   c->d_binom, c->bstride, 0, 1, ts));
                HIPCHK(launch_init_counters(st, p->d_queues, 1, nullptr, nullptr, 0, nullptr));
            }
            if (timing && single) HIPCHK(hipEventRecord(p->ev[2], st));
            if (s.pilot_n > 0 && item_cap == ~0ull)
                HIPCHK(launch_pilot(g.np2, g.np3, g.gk, std::min(g.grid, s.pilot_n / 4), st, tasks + i, 1,
                                    (unsigned long long)s.pilot_n, c->d_binom, c->bstride, g.tab_cap, g.kmax,
                                    g.stage_cap));
            HIPCHK(launch_scan(g.np2, g.np3, g.gk, g.grid, st, tasks + i, 1, std::min(s.n_items, item_cap),
                               p->d_queues + 1, c->d_binom, c->bstride, g.tab_cap, g.kmax, g.stage_cap, p->check));
            HIPCHK(launch_init_counters(st, p->d_queues + 1, 1, nullptr, nullptr, 0, nullptr));
            if (timing && single) HIPCHK(hipEventRecord(p->ev[3], st));
            HIPCHK(launch_merge(1, st, tasks + i, (Cand *)p->d_parts + (size_t)i * kMergeParts * kMaxTopK,
                                (Cand *)p->d_results + (size_t)i * kMaxTopK));
            HIPCHK(launch_finalize(1, s.desc.top_k, st, tasks + i, (const Cand *)p->d_results + (size_t)i * kMaxTopK,
                                   (const ResultLayout *)p->d_layout + i, (char *)p->d_out));
        }
    }
    if (p->arena) {
        // allocation-free plan (one scan): its result block to the caller's buffers
        const PlanScan &s = p->scans[0];
        HIPCHK(launch_scatter(st, (const char *)p->d_out + s.lay.offset, s.desc.top_k, s.desc.order, p->u_combos,
                              p->u_scores, p->u_tables, p->u_n));
        return EPI_OK;
    }
    HIPCHK(hipMemcpyAsync(p->h_out, p->d_out, (size_t)std::max<long long>(p->out_bytes, 256), hipMemcpyDeviceToHost, st));
    if (p->check)
        HIPCHK(hipMemcpyAsync((char *)p->h_out + std::max<long long>(p->out_bytes, 256), p->d_digest,
                              (size_t)nt * 16, hipMemcpyDeviceToHost, st));
    return EPI_OK;
}

int plan_run(Ctx *c, Plan *p, hipStream_t st, unsigned long long item_cap) {
    if (!st) st = c->stream;
    p->stream = st;
    p->timed = false;
    if (p->use_graph) {
        if (!p->exec) {
            hipStream_t cap;
            HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            int rc = plan_enqueue(c, p, cap, false, item_cap);
            hipGraph_t gr = nullptr;
            hipError_t e = hipStreamEndCapture(cap, &gr);
            (void)hipStreamDestroy(cap);
            if (rc) return rc;
            if (e != hipSuccess) return fail(EPI_EDEVICE, "graph capture: %s", hipGetErrorString(e));
            p->graph = gr;
            HIPCHK(hipGraphInstantiate(&p->exec, gr, nullptr, nullptr, 0));
        }
        HIPCHK(hipEventRecord(p->ev[0], st));
        HIPCHK(hipGraphLaunch(p->exec, st));
        HIPCHK(hipEventRecord(p->ev[4], st));
    } else {
        HIPCHK(hipEventRecord(p->ev[0], st));
        int rc = plan_enqueue(c, p, st, true, item_cap);
        if (rc) return rc;
        HIPCHK(hipEventRecord(p->ev[4], st));
        p->timed = p->scans.size() == 1;
    }
    p->ran = true;
    return EPI_OK;
}

int plan_wait(Plan *p) {
    if (!p->ran) return fail(EPI_ENOTREADY, "plan has not run");
    HIPCHK(hipEventSynchronize(p->ev[4]));
    return EPI_OK;
}

// Error bits of a dataset's packing (set by the device kernels): 1 a genotype
// outside {0,1,2}, 2 a phenotype outside {0,1}, 4 class sizes that differ
// from the dataset's, 8 an individual index out of range.
int pack_error(int bits) {
    return fail(EPI_EINVAL, "the dataset's last packing had invalid input (device check bits 0x%x:%s%s%s)", bits,
                (bits & 1) ? " genotype outside {0,1,2}" : "", (bits & 2) ? " phenotype outside {0,1}" : "",
                (bits & 12) ? " class sizes differ from the dataset's" : "");
}

int plan_results(Plan *p, int index, int capacity, int32_t *combos, float *scores, uint32_t *tables,
                 int32_t *n_written) {
    if (index < 0 || index >= (int)p->scans.size()) return fail(EPI_EINVAL, "scan index %d out of range", index);
    if (!p->ran) return fail(EPI_ENOTREADY, "scan has not run");
    hipError_t q = hipEventQuery(p->ev[4]);
    if (q == hipErrorNotReady) return fail(EPI_ENOTREADY, "scan not finished");
    if (q != hipSuccess) return fail(EPI_EDEVICE, "scan failed: %s", hipGetErrorString(q));
    if (capacity < 0 || !n_written) return fail(EPI_EINVAL, "bad capacity / n_written");
    const PlanScan &s = p->scans[index];
    const int K = s.desc.top_k, k = s.desc.order, cells = pow3i(k);
    const char *blk = (const char *)p->h_out + s.lay.offset;
    const int32_t nv = *(const int32_t *)blk;
    const int32_t perr = ((const int32_t *)blk)[1];
    if (perr) return pack_error(perr);
    const int32_t *hc = (const int32_t *)(blk + 16);
    const float *hs = (const float *)(blk + 16 + (size_t)K * k * 4);
    const uint32_t *ht = (const uint32_t *)(blk + 16 + (size_t)K * k * 4 + (size_t)K * 4);
    const int n = std::min(capacity, nv);
    if (n > 0 && (!combos || !scores)) return fail(EPI_EINVAL, "null combos/scores buffer");
    for (int r = 0; r < n; ++r) {
        memcpy(combos + (size_t)r * k, hc + (size_t)r * k, (size_t)k * 4);
        scores[r] = hs[r];
        if (tables) memcpy(tables + (size_t)r * 2 * cells, ht + (size_t)r * 2 * cells, (size_t)2 * cells * 4);
    }
    *n_written = n;
    return EPI_OK;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
void load_tune_cache(Ctx *c) {
    std::ifstream f(c->tune_path);
    std::string arch;
    int order, bucket, np;
    while (f >> arch >> order >> bucket >> np) {
        if (arch != c->arch) continue;
        if (np == EPI_BLOCK_SEGMENTED) c->seg_pins[TuneKey{order, bucket}] = 1;
        else c->tuned[TuneKey{order, bucket}] = np;
    }
}

static void save_tune_cache(Ctx *c) {
    if (c->tune_path.empty()) return;
    std::ofstream f(c->tune_path, std::ios::trunc);
    for (auto &kv : c->tuned) f << c->arch << " " << kv.first.order << " " << kv.first.bucket << " " << kv.second << "\n";
    for (auto &kv : c->seg_pins)
        f << c->arch << " " << kv.first.order << " " << kv.first.bucket << " " << EPI_BLOCK_SEGMENTED << "\n";
}

// Size bucket of a dataset for tuned choices: the power-of-two buckets of
// its 32-bit words per SNP row (both classes) and of its number of SNPs, as
// 64 x words bucket + SNP bucket.
int size_bucket(const Dataset *d) {
    const int words = (d->w4[0] + d->w4[1]) * 4;
    int wb = 0, mb = 0;
    while ((1 << wb) < words) ++wb;
    while ((1 << mb) < d->M) ++mb;
    return wb * 64 + mb;
}

// Combinations a kernel scores in items [a, b) of a scan: the valid triplets
// or pairs of each item's blocks (i < j < m, all below M), or the ranks of a
// per-combination item that are below C(M, k).
static unsigned long long valid_in_items(const PlanScan &s, unsigned long long a, unsigned long long b) {
    const long long M = s.ds->M;
    if (s.variant != kF2 && s.variant != kF3) {
        const unsigned long long per = 64ull * kGenRanksHost;
        const unsigned long long lo = std::min(a * per, s.n_combos), hi = std::min(b * per, s.n_combos);
        return hi - lo;
    }
    const int kind = item_kind(s.variant, s.np);
    const int np = s.np;
    auto clip = [](long long lo, long long hi) { return hi > lo ? hi - lo : 0LL; };  // size of [lo, hi)
    unsigned long long n = 0, at = 0;
    const long long G = item_groups(kind, (int)M, np);
    for (long long g = 0; g < G && at < b; ++g) {
        const ItemGroup gr = item_group(kind, (int)M, np, g);
        if (at + gr.count <= a) {
            at += gr.count;
            continue;
        }
        for (unsigned long long t = 0; t < gr.count && at < b; ++t, ++at) {
            if (at < a) continue;
            const unsigned long long dsc = item_at(gr, t);
            const long long j = (long long)(dsc >> 40), ib = (long long)((dsc >> 20) & 0xfffff),
                            mb = (long long)(dsc & 0xfffff);
            if (kind == kItemsF2) {
                const long long i0 = ib * np, m0 = i0 + 1 + mb * 64;
                for (long long i = i0; i < i0 + np && i <= M - 2; ++i) n += clip(std::max(m0, i + 1), std::min(m0 + 64, M));
            } else if (kind == kItemsF2M) {
                for (long long i = ib * 32; i < ib * 32 + 32 && i <= M - 2; ++i)
                    n += clip(std::max(mb * 32, i + 1), std::min(mb * 32 + 32, M));
            } else if (kind == kItemsF3) {
                const long long m0 = j + 1 + mb * 64;
                n += clip(ib * np, std::min(ib * np + np, j)) * clip(m0, std::min(m0 + 64, M));
            } else {
                n += clip(ib * 16, std::min(ib * 16 + 16, j)) * clip(std::max(mb * 32, j + 1), std::min(mb * 32 + 32, M));
            }
        }
    }
    return n;
}

// Candidate kernels of an order, by the block that pins them (order 4:
// kForceReducedCells for the reduced-cell kernel, which epi_set_prefix_block
// calls 0).
static std::vector<int> tune_candidates(const Dataset *ds, int order) {
    if (order == 2) {
        std::vector<int> v{2, 4, 8};
        if (ds->qa) v.push_back(kNpMfma);
        return v;
    }
    if (order == 3) {
        std::vector<int> v{1, 2, 4, 8};
        if (ds->qa) {
            v.push_back(kNpMfma);
            if (np3_usable(ds, kNpMfma2)) v.push_back(kNpMfma2);
        }
        return v;
    }
    std::vector<int> v;
    if (order == 4 && r4_fits(ds)) v.push_back(kForceReducedCells);
    v.push_back(EPI_BLOCK_ALL_CELLS);
    v.push_back(EPI_BLOCK_SEGMENTED);
    return v;
}

// Time each candidate kernel on slices spread over the whole work-item space
// of the dataset's own scan (kSlices contiguous runs at evenly spaced
// starts, each about 8 items per wave of its launch, so the launch's start
// and drain do not decide), normalised by the combinations those items score
// (counted on the host from the items), and keep the fastest per (order,
// size bucket).
int autotune(Ctx *c, int ds_id, int order, int *choice) {
    constexpr int kSlices = 8;
    Dataset *ds;
    epi_scan_desc d{ds_id, order, 16, 0};
    {
        std::lock_guard<std::mutex> g(c->mu);
        int rc = check_desc(c, d, &ds);
        if (rc) return rc;
    }
    const std::vector<int> cands = tune_candidates(ds, order);
    std::vector<std::pair<int, double>> report;
    double best_t = 1e30;
    int best = cands[0];
    for (int blk : cands) {
        Plan *p = nullptr;
        int rc = plan_build(c, &d, 1, false, false, &p, blk);
        if (rc) return rc;
        const PlanScan &s = p->scans[0];
        const unsigned long long total = s.n_items;
        const unsigned long long len = std::max<unsigned long long>(
            1, std::min<unsigned long long>(total / kSlices, (unsigned long long)p->groups[0].grid * 4 * 8));
        Task *staged = (Task *)((char *)p->h_stage + p->stage_layout_bytes);
        // slices are timed without the pilot pass (its items span the task)
        p->scans[0].pilot_n = 0;
        staged[0].pilot_n = 0;
        staged[0].pilot_first = 0;
        double best_rep = 1e30;
        for (int rep = 0; rep < 3 && !rc; ++rep) {
            double ms_sum = 0;
            unsigned long long valid = 0;
            for (int k = 0; k < kSlices && !rc; ++k) {
                const unsigned long long first = total > len ? (total - len) * (unsigned long long)k / (kSlices - 1) : 0;
                const unsigned long long n = std::min(len, total - first);
                staged[0].first_item = first;
                rc = plan_run(c, p, c->stream, n);
                if (!rc) rc = plan_wait(p);
                float ms = 0;
                if (!rc && hipEventElapsedTime(&ms, p->ev[2], p->ev[3]) == hipSuccess) ms_sum += ms;
                valid += valid_in_items(s, first, first + n);
                if (total <= len) break;
            }
            if (!rc && rep > 0 && valid) best_rep = std::min(best_rep, ms_sum * 1e6 / (double)valid);
        }
        plan_free(c, p);
        delete p;
        if (rc) return rc;
        report.emplace_back(order >= 4 && blk == kForceReducedCells ? 0 : blk, best_rep);
        if (best_rep < best_t) {
            best_t = best_rep;
            best = blk;
        }
    }
    const TuneKey key{order, size_bucket(ds)};
    {
        std::lock_guard<std::mutex> g(c->tune_mu);
        c->seg_pins.erase(key);
        c->tuned.erase(key);
        if (best == EPI_BLOCK_SEGMENTED) c->seg_pins[key] = 1;
        else if (order <= 3 || (order == 4 && best == EPI_BLOCK_ALL_CELLS && r4_fits(ds))) c->tuned[key] = best;
        c->tune_report[key] = report;
        save_tune_cache(c);
    }
    *choice = order >= 4 && best == kForceReducedCells ? 0 : best;
    return EPI_OK;
}

}  // namespace epi

// ===========================================================================
// C ABI
// ===========================================================================
using namespace epi;

#define CTX_OR_FAIL(ctx)                                                  \
    if (!(ctx)) return fail(EPI_EINVAL, "null context");                  \
    Ctx *C = as_ctx(ctx);                                                 \
    if (hipSetDevice(C->device) != hipSuccess) return fail(EPI_EDEVICE, "hipSetDevice failed");

extern "C" {

const char *epi_last_error(void) { return last_error(); }

const char *epi_version(void) { return "epi-mi355x 0.2 (gfx950)"; }

int epi_create(int32_t device, uint64_t hbm_budget_bytes, epi_ctx **out) {
    clear_error();
    if (!out) return fail(EPI_EINVAL, "null out");
    auto c = std::make_unique<Ctx>();
    int rc = ctx_init(c.get(), device, hbm_budget_bytes);
    if (rc) {
        c->alloc.destroy();
        return rc;
    }
    *out = reinterpret_cast<epi_ctx *>(c.release());
    return EPI_OK;
}

int epi_destroy(epi_ctx *ctx) {
    clear_error();
    if (!ctx) return EPI_OK;
    Ctx *C = as_ctx(ctx);
    (void)hipSetDevice(C->device);
    server_shutdown_all(C);
    (void)hipDeviceSynchronize();
    for (auto &kv : C->plans) plan_free(C, kv.second.get());
    C->plans.clear();
    pools_free(C);
    C->item_tables.clear();
    for (auto &kv : C->datasets) ds_free(C, kv.second.get());
    C->datasets.clear();
    C->alloc.destroy();
    if (C->stream) (void)hipStreamDestroy(C->stream);
    delete C;
    return EPI_OK;
}

int epi_memory(epi_ctx *ctx, uint64_t *used_bytes, uint64_t *budget_bytes) {
    clear_error();
    CTX_OR_FAIL(ctx);
    if (used_bytes) *used_bytes = C->alloc.used;
    if (budget_bytes) *budget_bytes = C->alloc.budget;
    return EPI_OK;
}

int epi_load_genotypes(epi_ctx *ctx, const uint8_t *geno, int64_t ld, const uint8_t *pheno, int32_t M, int32_t N,
                       int32_t *dataset_id) {
    clear_error();
    CTX_OR_FAIL(ctx);
    if (!geno || !pheno || !dataset_id) return fail(EPI_EINVAL, "null argument");
    if (M < 1 || N < 2 || ld < N) return fail(EPI_EINVAL, "bad shape M=%d N=%d ld=%lld", M, N, (long long)ld);
    // genotype check on the host (the device kernel checks too)
    for (int32_t s = 0; s < M; ++s) {
        const uint8_t *row = geno + (size_t)s * ld;
        for (int32_t i = 0; i < N; ++i)
            if (row[i] > 2) return fail(EPI_EINVAL, "genotype of SNP %d individual %d is %d", s, i, row[i]);
    }
    std::vector<uint8_t> hp(pheno, pheno + N);
    void *dg = nullptr, *dp = nullptr;
    int rc = C->alloc.alloc((size_t)M * N, &dg);
    if (!rc) rc = C->alloc.alloc((size_t)N, &dp);
    if (!rc) {
        hipError_t e = hipMemcpy2DAsync(dg, N, geno, ld, N, M, hipMemcpyHostToDevice, C->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(dp, pheno, N, hipMemcpyHostToDevice, C->stream);
        if (e != hipSuccess) rc = fail(EPI_EDEVICE, "upload: %s", hipGetErrorString(e));
    }
    if (!rc) rc = load_common(C, (const uint8_t *)dg, N, (const uint8_t *)dp, hp, M, N, C->stream, dataset_id);
    (void)hipStreamSynchronize(C->stream);
    C->alloc.release(dg);
    C->alloc.release(dp);
    return rc;
}

int epi_load_genotypes_device(epi_ctx *ctx, const uint8_t *d_geno, int64_t ld, const uint8_t *d_pheno, int32_t M,
                              int32_t N, void *stream, int32_t *dataset_id) {
    clear_error();
    CTX_OR_FAIL(ctx);
    if (!d_geno || !d_pheno || !dataset_id) return fail(EPI_EINVAL, "null argument");
    if (M < 1 || N < 2 || ld < N) return fail(EPI_EINVAL, "bad shape M=%d N=%d ld=%lld", M, N, (long long)ld);
    hipStream_t st = stream ? (hipStream_t)stream : C->stream;
    std::vector<uint8_t> hp(N);
    HIPCHK(hipMemcpyAsync(hp.data(), d_pheno, N, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return load_common(C, d_geno, ld, d_pheno, hp, M, N, st, dataset_id);
}

int epi_repack_device(epi_ctx *ctx, int32_t dataset_id, const uint8_t *d_geno, int64_t ld, const uint8_t *d_pheno,
                      void *stream) {
    clear_error();
    CTX_OR_FAIL(ctx);
    auto it = C->datasets.find(dataset_id);
    if (it == C->datasets.end()) return fail(EPI_ENOTFOUND, "unknown dataset %d", dataset_id);
    Dataset *d = it->second.get();
    if (!d_geno || !d_pheno || ld < d->N) return fail(EPI_EINVAL, "bad repack arguments");
    hipStream_t st = stream ? (hipStream_t)stream : C->stream;
    return ds_pack(d, d_geno, ld, d_pheno, st);
}

int epi_unload(epi_ctx *ctx, int32_t dataset_id) {
    clear_error();
    CTX_OR_FAIL(ctx);
    std::unique_ptr<Dataset> d;
    {
        std::lock_guard<std::mutex> g(C->mu);
        auto it = C->datasets.find(dataset_id);
        if (it == C->datasets.end()) return fail(EPI_ENOTFOUND, "unknown dataset %d", dataset_id);
        const int users = it->second->users.load();
        if (users > 0)
            return fail(EPI_EINVAL, "dataset %d is read by %d queued or running server requests", dataset_id, users);
        d = std::move(it->second);
        C->datasets.erase(it);
    }
    (void)hipDeviceSynchronize();
    ds_free(C, d.get());
    return EPI_OK;
}

int epi_dataset_info(epi_ctx *ctx, int32_t dataset_id, int32_t *M, int32_t *N, int32_t *n_cases,
                     uint64_t *device_bytes) {
    clear_error();
    CTX_OR_FAIL(ctx);
    auto it = C->datasets.find(dataset_id);
    if (it == C->datasets.end()) return fail(EPI_ENOTFOUND, "unknown dataset %d", dataset_id);
    const Dataset *d = it->second.get();
    if (M) *M = d->M;
    if (N) *N = d->N;
    if (n_cases) *n_cases = d->n_case;
    if (device_bytes) *device_bytes = d->bytes;
    return EPI_OK;
}

static int register_plan(Ctx *C, Plan *p, int32_t *scan_ids) {
    std::lock_guard<std::mutex> g(C->mu);
    p->id = C->next_id++;
    for (size_t i = 0; i < p->scans.size(); ++i) {
        const int sid = C->next_id++;
        C->scan_index[sid] = ScanRef{p->id, (int)i};
        p->scans[i].scan_id = sid;
        if (scan_ids) scan_ids[i] = sid;
        p->live_scans++;
    }
    C->plans[p->id] = std::unique_ptr<Plan>(p);
    return p->id;
}

static Plan *plan_of_scan(Ctx *C, int32_t scan_id, int *index) {
    auto it = C->scan_index.find(scan_id);
    if (it == C->scan_index.end()) return nullptr;
    auto pit = C->plans.find(it->second.plan);
    if (pit == C->plans.end()) return nullptr;
    *index = it->second.index;
    return pit->second.get();
}

int epi_scan(epi_ctx *ctx, int32_t dataset_id, int32_t order, int32_t top_k, void *stream, int32_t *scan_id) {
    clear_error();
    CTX_OR_FAIL(ctx);
    if (!scan_id) return fail(EPI_EINVAL, "null scan_id");
    epi_scan_desc d{dataset_id, order, top_k, 0};
    Plan *p = nullptr;
    int rc = plan_build(C, &d, 1, false, false, &p, 0);
    if (rc) return rc;
    register_plan(C, p, scan_id);
    p->transient = true;
    return plan_run(C, p, (hipStream_t)stream, ~0ull);
}

int epi_scan_check(epi_ctx *ctx, int32_t dataset_id, int32_t order, int32_t top_k, void *stream, int32_t *scan_id) {
    clear_error();
    CTX_OR_FAIL(ctx);
    if (!scan_id) return fail(EPI_EINVAL, "null scan_id");
    epi_scan_desc d{dataset_id, order, top_k, 0};
    Plan *p = nullptr;
    int rc = plan_build(C, &d, 1, false, false, &p, 0, true);
    if (rc) return rc;
    register_plan(C, p, scan_id);
    p->transient = true;
    return plan_run(C, p, (hipStream_t)stream, ~0ull);
}

int epi_scan_digest(epi_ctx *ctx, int32_t scan_id, uint64_t *n_scored, uint64_t *digest) {
    clear_error();
    CTX_OR_FAIL(ctx);
    int idx;
    Plan *p = plan_of_scan(C, scan_id, &idx);
    if (!p) return fail(EPI_ENOTFOUND, "unknown scan %d", scan_id);
    if (!p->check) return fail(EPI_EINVAL, "scan %d was not started by epi_scan_check", scan_id);
    if (!n_scored || !digest) return fail(EPI_EINVAL, "null output");
    if (!p->ran) return fail(EPI_ENOTREADY, "scan has not run");
    hipError_t q = hipEventQuery(p->ev[4]);
    if (q == hipErrorNotReady) return fail(EPI_ENOTREADY, "scan not finished");
    if (q != hipSuccess) return fail(EPI_EDEVICE, "scan failed: %s", hipGetErrorString(q));
    const unsigned long long *w =
        (const unsigned long long *)((const char *)p->h_out + std::max<long long>(p->out_bytes, 256)) + 2 * idx;
    *n_scored = w[0];
    *digest = w[1];
    return EPI_OK;
}

int epi_scan_noalloc(epi_ctx *ctx, int32_t dataset_id, int32_t order, int32_t top_k, void *stream,
                     int32_t *d_combos, float *d_scores, uint32_t *d_tables, int32_t *d_n) {
    clear_error();
    CTX_OR_FAIL(ctx);
    if (!d_combos || !d_scores || !d_n) return fail(EPI_EINVAL, "null output buffer");
    epi_scan_desc d{dataset_id, order, top_k, 0};
    const PlanArena arena{C->scratch, kScratchBytes};
    Plan *p = nullptr;
    int rc = plan_build(C, &d, 1, false, false, &p, 0, false, &arena);
    if (rc) return rc;
    std::unique_ptr<Plan> hold(p);
    p->u_combos = d_combos;
    p->u_scores = d_scores;
    p->u_tables = d_tables;
    p->u_n = d_n;
    rc = plan_enqueue(C, p, stream ? (hipStream_t)stream : C->stream, false, ~0ull);
    plan_free(C, p);  // host state only: none of its device buffers came from an allocator
    return rc;
}

int epi_scan_batch(epi_ctx *ctx, const epi_scan_desc *descs, int32_t n, void *stream, int32_t *scan_ids) {
    clear_error();
    CTX_OR_FAIL(ctx);
    if (!descs || !scan_ids || n < 1) return fail(EPI_EINVAL, "bad batch arguments");
    Plan *p = nullptr;
    int rc = plan_build(C, descs, n, true, true, &p, 0);
    if (rc) return rc;
    register_plan(C, p, scan_ids);
    p->transient = true;
    return plan_run(C, p, (hipStream_t)stream, ~0ull);
}

int epi_scan_orders(epi_ctx *ctx, int32_t dataset_id, int32_t max_order, int32_t top_k, void *stream,
                    int32_t *scan_ids) {
    clear_error();
    CTX_OR_FAIL(ctx);
    if (!scan_ids) return fail(EPI_EINVAL, "null scan_ids");
    if (max_order < EPI_MIN_ORDER) return fail(EPI_EINVAL, "max_order %d < %d", max_order, EPI_MIN_ORDER);
    if (max_order > EPI_MAX_ORDER) return fail(EPI_EUNSUPPORTED, "max_order %d > %d", max_order, EPI_MAX_ORDER);
    std::vector<epi_scan_desc> descs;
    for (int o = EPI_MIN_ORDER; o <= max_order; ++o) descs.push_back(epi_scan_desc{dataset_id, o, top_k, 0});
    return epi_scan_batch(ctx, descs.data(), (int32_t)descs.size(), stream, scan_ids);
}

int epi_query(epi_ctx *ctx, int32_t scan_id, int32_t *done) {
    clear_error();
    CTX_OR_FAIL(ctx);
    int idx;
    Plan *p = plan_of_scan(C, scan_id, &idx);
    if (!p) return fail(EPI_ENOTFOUND, "unknown scan %d", scan_id);
    if (!done) return fail(EPI_EINVAL, "null done");
    if (!p->ran) {
        *done = 0;
        return EPI_OK;
    }
    hipError_t q = hipEventQuery(p->ev[4]);
    if (q != hipSuccess && q != hipErrorNotReady) return fail(EPI_EDEVICE, "%s", hipGetErrorString(q));
    *done = q == hipSuccess ? 1 : 0;
    return EPI_OK;
}

int epi_wait(epi_ctx *ctx, int32_t scan_id) {
    clear_error();
    CTX_OR_FAIL(ctx);
    int idx;
    Plan *p = plan_of_scan(C, scan_id, &idx);
    if (!p) return fail(EPI_ENOTFOUND, "unknown scan %d", scan_id);
    return plan_wait(p);
}

int epi_results(epi_ctx *ctx, int32_t scan_id, int32_t capacity, int32_t *combos, float *scores, uint32_t *tables,
                int32_t *n_written) {
    clear_error();
    CTX_OR_FAIL(ctx);
    int idx;
    Plan *p = plan_of_scan(C, scan_id, &idx);
    if (!p) return fail(EPI_ENOTFOUND, "unknown scan %d", scan_id);
    return plan_results(p, idx, capacity, combos, scores, tables, n_written);
}

int epi_scan_timing(epi_ctx *ctx, int32_t scan_id, float ms[4]) {
    clear_error();
    CTX_OR_FAIL(ctx);
    int idx;
    Plan *p = plan_of_scan(C, scan_id, &idx);
    if (!p) return fail(EPI_ENOTFOUND, "unknown scan %d", scan_id);
    if (!ms) return fail(EPI_EINVAL, "null ms");
    int rc = plan_wait(p);
    if (rc) return rc;
    for (int i = 0; i < 4; ++i) ms[i] = -1.0f;
    HIPCHK(hipEventElapsedTime(&ms[0], p->ev[0], p->ev[4]));
    if (p->timed) {
        if (p->scans[0].desc.order == 3) HIPCHK(hipEventElapsedTime(&ms[1], p->ev[1], p->ev[2]));
        HIPCHK(hipEventElapsedTime(&ms[2], p->ev[2], p->ev[3]));
        HIPCHK(hipEventElapsedTime(&ms[3], p->ev[3], p->ev[4]));
    }
    return EPI_OK;
}

int epi_scan_info(epi_ctx *ctx, int32_t scan_id, uint64_t *n_combinations, int32_t *variant, int32_t *prefix_block) {
    clear_error();
    CTX_OR_FAIL(ctx);
    int idx;
    Plan *p = plan_of_scan(C, scan_id, &idx);
    if (!p) return fail(EPI_ENOTFOUND, "unknown scan %d", scan_id);
    const PlanScan &s = p->scans[idx];
    if (n_combinations) *n_combinations = s.n_combos;
    if (variant) *variant = s.variant;
    if (prefix_block) *prefix_block = s.np;
    return EPI_OK;
}

int epi_release(epi_ctx *ctx, int32_t scan_id) {
    clear_error();
    CTX_OR_FAIL(ctx);
    std::unique_ptr<Plan> dead;
    {
        std::lock_guard<std::mutex> g(C->mu);
        auto it = C->scan_index.find(scan_id);
        if (it == C->scan_index.end()) return fail(EPI_ENOTFOUND, "unknown scan %d", scan_id);
        auto pit = C->plans.find(it->second.plan);
        C->scan_index.erase(it);
        if (pit == C->plans.end()) return EPI_OK;
        Plan *p = pit->second.get();
        if (--p->live_scans <= 0 && p->transient) {
            dead = std::move(pit->second);
            C->plans.erase(pit);
        }
    }
    if (dead) {
        if (dead->ran) (void)hipEventSynchronize(dead->ev[4]);
        plan_free(C, dead.get());
    }
    return EPI_OK;
}

int epi_batch_create(epi_ctx *ctx, const epi_scan_desc *descs, int32_t n, int32_t persistent, int32_t use_graph,
                     int32_t *batch_id) {
    clear_error();
    CTX_OR_FAIL(ctx);
    if (!descs || !batch_id || n < 1) return fail(EPI_EINVAL, "bad batch arguments");
    Plan *p = nullptr;
    int rc = plan_build(C, descs, n, persistent != 0, use_graph != 0, &p, 0);
    if (rc) return rc;
    *batch_id = register_plan(C, p, nullptr);
    p->transient = false;
    return EPI_OK;
}

static Plan *batch_of(Ctx *C, int32_t id) {
    auto it = C->plans.find(id);
    if (it == C->plans.end() || it->second->transient) return nullptr;
    return it->second.get();
}

int epi_batch_run(epi_ctx *ctx, int32_t batch_id, void *stream) {
    clear_error();
    CTX_OR_FAIL(ctx);
    Plan *p = batch_of(C, batch_id);
    if (!p) return fail(EPI_ENOTFOUND, "unknown batch %d", batch_id);
    for (auto &s : p->scans)
        if (!C->datasets.count(s.desc.dataset_id)) return fail(EPI_ENOTFOUND, "dataset %d was unloaded", s.desc.dataset_id);
    return plan_run(C, p, (hipStream_t)stream, ~0ull);
}

int epi_batch_wait(epi_ctx *ctx, int32_t batch_id) {
    clear_error();
    CTX_OR_FAIL(ctx);
    Plan *p = batch_of(C, batch_id);
    if (!p) return fail(EPI_ENOTFOUND, "unknown batch %d", batch_id);
    return plan_wait(p);
}

int epi_batch_results(epi_ctx *ctx, int32_t batch_id, int32_t index, int32_t capacity, int32_t *combos, float *scores,
                      uint32_t *tables, int32_t *n_written) {
    clear_error();
    CTX_OR_FAIL(ctx);
    Plan *p = batch_of(C, batch_id);
    if (!p) return fail(EPI_ENOTFOUND, "unknown batch %d", batch_id);
    return plan_results(p, index, capacity, combos, scores, tables, n_written);
}

int epi_batch_timing(epi_ctx *ctx, int32_t batch_id, float *ms) {
    clear_error();
    CTX_OR_FAIL(ctx);
    Plan *p = batch_of(C, batch_id);
    if (!p) return fail(EPI_ENOTFOUND, "unknown batch %d", batch_id);
    if (!ms) return fail(EPI_EINVAL, "null ms");
    int rc = plan_wait(p);
    if (rc) return rc;
    HIPCHK(hipEventElapsedTime(ms, p->ev[0], p->ev[4]));
    return EPI_OK;
}

int epi_batch_destroy(epi_ctx *ctx, int32_t batch_id) {
    clear_error();
    CTX_OR_FAIL(ctx);
    std::unique_ptr<Plan> dead;
    {
        std::lock_guard<std::mutex> g(C->mu);
        auto it = C->plans.find(batch_id);
        if (it == C->plans.end() || it->second->transient) return fail(EPI_ENOTFOUND, "unknown batch %d", batch_id);
        dead = std::move(it->second);
        C->plans.erase(it);
    }
    if (dead->ran) (void)hipEventSynchronize(dead->ev[4]);
    plan_free(C, dead.get());
    return EPI_OK;
}

int epi_set_prefix_block(epi_ctx *ctx, int32_t dataset_id, int32_t order, int32_t block) {
    clear_error();
    CTX_OR_FAIL(ctx);
    Dataset *d;
    {
        std::lock_guard<std::mutex> g(C->mu);
        auto it = C->datasets.find(dataset_id);
        if (it == C->datasets.end()) return fail(EPI_ENOTFOUND, "unknown dataset %d", dataset_id);
        d = it->second.get();
    }
    const bool ok2 = order == 2 && (block == 2 || block == 4 || block == 8 || block == kNpMfma);
    const bool ok3 = order == 3 && (block == 1 || block == 2 || block == 4 || block == 8 || is_mfma_np(block));
    const bool any = order >= EPI_MIN_ORDER && order <= EPI_MAX_ORDER && (block == 0 || block == EPI_BLOCK_SEGMENTED);
    const bool all4 = order >= 4 && order <= EPI_MAX_ORDER && block == EPI_BLOCK_ALL_CELLS;
    if (!ok2 && !ok3 && !any && !all4)
        return fail(EPI_EINVAL, "prefix block %d is not a kernel of order %d", block, order);
    if ((block == kNpMfma || block == kNpMfma2) && !d->qa)
        return fail(EPI_EUNSUPPORTED, "dataset %d has no matrix-core operands (2^22 individuals or more)", dataset_id);
    if (block == kNpMfma2 && !np3_usable(d, block))
        return fail(EPI_EUNSUPPORTED,
                    "dataset %d: %d cases and %d controls do not fit one accumulator (4 cases + controls 2^T < 2^24)",
                    dataset_id, d->n_case, d->n_ctrl);
    if (block == kNpMfmaI8) {
        if (d->N >= (1 << 22))
            return fail(EPI_EUNSUPPORTED, "dataset %d: 2^22 individuals or more for the integer kernel", dataset_id);
        int rc = ds_ensure_i8(C, d);
        if (rc) return rc;
    }
    {
        std::lock_guard<std::mutex> g(C->tune_mu);
        const TuneKey key{order, size_bucket(d)};
        if (block == EPI_BLOCK_SEGMENTED) {
            C->seg_pins[key] = 1;
        } else if (block == 0) {
            C->seg_pins.erase(key);
            C->tuned.erase(key);
        } else {
            C->seg_pins.erase(key);
            C->tuned[key] = block;
        }
    }
    return EPI_OK;
}

// The steps of the method as separate passes (genotype rows, contingency
// tables, MI) over a device list of combinations or tables; synchronous.
static int run_function(epi_ctx *ctx, int fn, int32_t dataset_id, int32_t order, const int32_t *d_combos,
                        const uint32_t *d_tables, uint64_t n, void *d_out, float *kernel_ms) {
    clear_error();
    CTX_OR_FAIL(ctx);
    Dataset *d;
    {
        std::lock_guard<std::mutex> g(C->mu);
        auto it = C->datasets.find(dataset_id);
        if (it == C->datasets.end()) return fail(EPI_ENOTFOUND, "unknown dataset %d", dataset_id);
        d = it->second.get();
    }
    const int lo = fn == 0 ? 1 : EPI_MIN_ORDER;
    if (order < lo || order > EPI_MAX_ORDER)
        return fail(EPI_EINVAL, "order %d outside %d .. %d", order, lo, EPI_MAX_ORDER);
    if (kernel_ms) *kernel_ms = 0.f;
    if (n == 0) return EPI_OK;
    if (!d_out || (fn < 2 && !d_combos) || (fn == 2 && !d_tables)) return fail(EPI_EINVAL, "null buffer");
    const unsigned long long words = (unsigned long long)(d->w4[0] + d->w4[1]) * 4;
    const unsigned long long threads = fn == 0 ? n * words * (order >= 5 ? 9 : 1) : n;
    const unsigned long long want = (threads + 255) / 256;
    // MI stages its n ln n table per workgroup: fewer, longer-lived workgroups
    const int grid = (int)std::min<unsigned long long>(want, (unsigned long long)C->n_cu * (fn == 2 ? 8 : 64));
    void *d_err = nullptr;
    int rc = C->alloc.alloc(256, &d_err);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((rc = event_get(C, &e0)) || (rc = event_get(C, &e1))) {
        event_put(C, e0);
        C->alloc.release(d_err);
        return rc;
    }
    int h_err = 0;
    hipError_t he = hipMemsetAsync(d_err, 0, sizeof(int), C->stream);
    if (he == hipSuccess) he = hipEventRecord(e0, C->stream);
    if (he == hipSuccess)
        he = launch_function(fn, order, C->stream, d->view, d_combos, d_tables, n, d_out, (int *)d_err, grid,
                             d->score_const);
    if (he == hipSuccess) he = hipEventRecord(e1, C->stream);
    if (he == hipSuccess) he = hipMemcpyAsync(&h_err, d_err, sizeof(int), hipMemcpyDeviceToHost, C->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(C->stream);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    event_put(C, e0);
    event_put(C, e1);
    C->alloc.release(d_err);
    if (he != hipSuccess) return fail(EPI_EDEVICE, "device error: %s", hipGetErrorString(he));
    if (kernel_ms) *kernel_ms = ms;
    if (h_err)
        return fail(EPI_EINVAL, fn == 2 ? "a table does not fit the dataset's class sizes"
                                        : "a SNP index outside [0, %d)", d->M);
    return EPI_OK;
}

int epi_genotype_tables(epi_ctx *ctx, int32_t dataset_id, int32_t order, const int32_t *d_combos, uint64_t n,
                        uint32_t *d_rows, float *kernel_ms) {
    return run_function(ctx, 0, dataset_id, order, d_combos, nullptr, n, d_rows, kernel_ms);
}

int epi_contingency_tables(epi_ctx *ctx, int32_t dataset_id, int32_t order, const int32_t *d_combos, uint64_t n,
                           uint32_t *d_tables, float *kernel_ms) {
    return run_function(ctx, 1, dataset_id, order, d_combos, nullptr, n, d_tables, kernel_ms);
}

int epi_mutual_information(epi_ctx *ctx, int32_t dataset_id, int32_t order, const uint32_t *d_tables, uint64_t n,
                           double *d_mi, float *kernel_ms) {
    return run_function(ctx, 2, dataset_id, order, nullptr, d_tables, n, d_mi, kernel_ms);
}

int epi_autotune_report(epi_ctx *ctx, int32_t dataset_id, int32_t order, int32_t capacity, int32_t *blocks,
                        double *ns_per_combination, int32_t *n_candidates) {
    clear_error();
    CTX_OR_FAIL(ctx);
    if (!n_candidates || capacity < 0 || (capacity > 0 && (!blocks || !ns_per_combination)))
        return fail(EPI_EINVAL, "bad report buffers");
    Dataset *d;
    {
        std::lock_guard<std::mutex> g(C->mu);
        auto it = C->datasets.find(dataset_id);
        if (it == C->datasets.end()) return fail(EPI_ENOTFOUND, "unknown dataset %d", dataset_id);
        d = it->second.get();
    }
    std::lock_guard<std::mutex> g(C->tune_mu);
    auto it = C->tune_report.find(TuneKey{order, size_bucket(d)});
    if (it == C->tune_report.end()) return fail(EPI_ENOTFOUND, "no autotune of order %d for this size bucket", order);
    const int n = (int)it->second.size();
    for (int i = 0; i < std::min(n, capacity); ++i) {
        blocks[i] = it->second[i].first;
        ns_per_combination[i] = it->second[i].second;
    }
    *n_candidates = n;
    return EPI_OK;
}

int epi_autotune(epi_ctx *ctx, int32_t dataset_id, int32_t order, int32_t *choice) {
    clear_error();
    CTX_OR_FAIL(ctx);
    if (!choice) return fail(EPI_EINVAL, "null choice");
    return autotune(C, dataset_id, order, choice);
}

}  // extern "C"
