// Host-side state of the runtime (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/epi.h"
#include "epi_internal.hpp"

namespace epi {

constexpr int kBinomN = 65537;     // binomial table columns (n = 0 .. 65536)
constexpr int kGenRanksHost = 4;   // ranks per lane of the per-combination kernel
constexpr size_t kScratchBytes = EPI_NOALLOC_SCRATCH_BYTES;  // scratch array of allocation-free scans
// plan_build's forced kernel for order 4: the reduced-cell kernel (the
// blocks of the C ABI select the others)
constexpr int kForceReducedCells = 1;

int fail(int code, const char *fmt, ...);
void clear_error();
const char *last_error();

// Caching device allocator: freed blocks are kept per rounded size and
// reused; `used` (live bytes) may not exceed `budget`.
struct DevAlloc {
    std::mutex mu;
    std::multimap<size_t, void *> free_;
    std::map<void *, size_t> live;
    uint64_t used = 0, cached = 0, peak = 0, budget = 0;
    int alloc(size_t bytes, void **out);
    void release(void *p);
    void trim();
    void trim_locked();
    void destroy();
};

struct Dataset {
    int id = 0;
    int M = 0, N = 0, n_case = 0, n_ctrl = 0, Mp = 0, shift = 0;
    int w4[2] = {0, 0};
    void *masks = nullptr, *single = nullptr, *tlog = nullptr, *itab = nullptr, *idx = nullptr, *err = nullptr;
    int ks[2] = {0, 0};                   // 64-individual steps per class of qa / qb
    void *qa = nullptr, *qb = nullptr;    // matrix-core operand copies (null: order 3 by popcount only)
    int ks8[2] = {0, 0};                  // 32-individual steps per class of qa8 / qb8
    void *qa8 = nullptr, *qb8 = nullptr;  // integer operand copies, built on first selection
    long long score_const = 0;
    int tq = 0;
    uint64_t bytes = 0;
    DsView view{};
    // server requests (queued or admitted) that read this dataset; epi_unload
    // refuses while any do
    std::atomic<int> users{0};
};

struct PlanScan {
    epi_scan_desc desc{};
    Dataset *ds = nullptr;
    int variant = 0, np = 0;
    unsigned long long n_combos = 0, n_items = 0;
    const void *items = nullptr;  // cached per-item descriptors (owned by the context)
    // order 3: pair sub-table pass
    int emit_np = 0, emit_task = -1;
    unsigned long long emit_items = 0;
    const void *emit_items_d = nullptr;
    void *pairs = nullptr;
    // order 4 by reduced cells: triplet sub-table pass
    void *triples = nullptr;
    int t3_task = -1;
    void *seg = nullptr;  // segmented variant: the launch's per-wave table blocks
    unsigned long long t3_items = 0;
    const void *t3_items_d = nullptr;
    void *cand = nullptr;
    unsigned cand_cap = 0;
    ResultLayout lay{};
    int scan_id = -1;
    // matrix-core order 3 and reduced-cell order 4: pilot pass over items
    // pilot_first .. pilot_first + pilot_n - 1 (pilot_n 0: none)
    int pilot_n = 0;
    unsigned long long pilot_first = 0;
};

struct LaunchGroup {
    int np2 = 0, np3 = 0, gk = 0, grid = 1;  // grid: 4-wave workgroups
    int tab_cap = 0;                         // LDS screening-table entries (0: none)
    int kmax = 1, stage_cap = 0;
    int task_off = 0;  // first task of the group in the plan's task array
    std::vector<int> scans;
    unsigned long long total_items = 0;
    unsigned long long pilot_total = 0;  // pilot items of the group's tasks (0: no pilot launch)
};

struct Plan {
    int id = 0;
    bool persistent = false, use_graph = false, transient = false, ran = false, timed = false;
    bool check = false;  // checking launch: the main passes also count and digest every combination
    int live_scans = 0;
    std::vector<PlanScan> scans;
    std::vector<LaunchGroup> groups;
    int n_emit = 0, emit_grid = 1, emit_stage = 0, n_queues = 0;
    int emit_kmax = 1;  // best-K list entries per wave of the pair-pass launch (order-2 scans scored there)
    constexpr static int kTabMax = 16386;  // screening-table entries that may go to LDS
    unsigned long long emit_total = 0;
    int n_t3 = 0, t3_grid = 1, t3_stage = 0;  // triplet sub-table pass (order 4 by reduced cells)
    unsigned long long t3_total = 0;
    void *d_tasks = nullptr, *d_counters = nullptr, *d_results = nullptr, *d_layout = nullptr, *d_out = nullptr;
    void *d_parts = nullptr;
    void *h_out = nullptr;                // pinned, from the context's pool
    size_t h_out_cap = 0;
    void *h_stage = nullptr;              // pinned copies of the layout and task arrays, uploaded by every run
    size_t h_stage_cap = 0, stage_layout_bytes = 0, stage_tasks_bytes = 0;
    unsigned long long *d_queues = nullptr, *d_thr = nullptr;
    unsigned long long *d_digest = nullptr;  // check: 2 words per scan, zeroed with the queues
    unsigned *d_cand_count = nullptr;
    unsigned *d_hist = nullptr;  // kHistWords per scan
    long long out_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hipStream_t stream = nullptr;
    // Allocation-free plans (epi_scan_noalloc): every device buffer is carved
    // from the device's scratch array, the task and layout arrays reach the
    // device in kernel arguments (no copy from host memory), descriptor
    // tables the context has not cached yet are written into the scratch by
    // the run, and there are no events.  The results go to the caller's
    // device buffers.
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    struct ItemGen {
        int kind, M, np;
        void *dst;
    };
    std::vector<ItemGen> item_gens;  // descriptor tables the run writes first
    std::vector<char> h_stage_mem;   // host copy of the layout and task arrays
    int32_t *u_combos = nullptr, *u_n = nullptr;
    float *u_scores = nullptr;
    uint32_t *u_tables = nullptr;
};

struct ScanRef {
    int plan = 0, index = 0;
};

struct TuneKey {
    int order, bucket;
    bool operator<(const TuneKey &o) const { return order != o.order ? order < o.order : bucket < o.bucket; }
};

struct Server;

// Work-item descriptor table of one (variant, M, prefix block) shape.
struct ItemTable {
    void *d = nullptr;
    unsigned long long n = 0;
};

struct Ctx {
    int device = 0, n_cu = 1, bstride = 0;
    std::string arch;
    hipStream_t stream = nullptr;
    DevAlloc alloc;
    unsigned long long *d_binom = nullptr;
    std::mutex mu;
    int next_id = 1;
    std::map<int, std::unique_ptr<Dataset>> datasets;
    std::map<int, std::unique_ptr<Plan>> plans;
    std::map<int, ScanRef> scan_index;
    std::mutex tune_mu;
    std::map<TuneKey, int> tuned;
    std::map<TuneKey, int> seg_pins;  // (order, bucket) pinned to the segmented variant
    // the last autotune of each (order, bucket): candidate block, ns per valid combination
    std::map<TuneKey, std::vector<std::pair<int, double>>> tune_report;
    std::string tune_path;
    std::map<int, std::shared_ptr<Server>> servers;
    std::mutex items_mu;
    std::map<std::tuple<int, int, int>, ItemTable> item_tables;
    // pinned host buffers (by capacity) and events kept for later plans:
    // freeing pinned memory and events per scan costs more than the scan's
    // own host work
    std::mutex pool_mu;
    std::multimap<size_t, void *> host_pool;
    size_t host_pool_bytes = 0;
    std::vector<hipEvent_t> event_pool;
    char *scratch = nullptr;  // this device's scratch array (allocation-free scans)
};

// kernel launchers (kernels.hip)
hipError_t launch_pilot(int np2, int np3, int gk, int grid, hipStream_t st, const Task *tasks, int n_tasks,
                        unsigned long long total, const unsigned long long *binom, int bstride, int tab_cap, int kmax,
                        int stage_cap);
// Pilot items of a task (a multiple of 4; 0: none): up to one per wave of its
// launch, when the task has at least 32 items per pilot item and the pilot
// counts can reach a bound (twice top_k of them), and its screening table
// fits the launch's LDS table (tab_cap entries).
int pilot_items_for(int variant, int np, unsigned long long n_items, int top_k, int N, int tab_cap, int waves);
// 4-wave workgroups per CU of a scan kernel instantiation (VGPRs and LDS:
// screening-table entries, best-K list entries per wave, staged rows).
int wgs_per_cu(int np2, int np3, int gk, int tab_cap, int kmax, int stage_cap);
// Best-K list entries per wave of a launch group: room for batched insertion
// (list_cap) unless that costs workgroups per CU, else top_k.
bool table_lowers_occupancy(const Dataset *d, int variant, int np, int order, int top_k);
int group_list_cap(int np2, int np3, int gk, int tab_cap, int top_k, int stage_cap);
hipError_t launch_scan(int np2, int np3, int gk, int grid, hipStream_t st, const Task *tasks, int n_tasks,
                       unsigned long long total_items, unsigned long long *queue, const unsigned long long *binom,
                       int bstride, int tab_cap, int kmax, int stage_cap, bool check = false);
size_t scan_lds_bytes(int tab_cap, int kmax, int stage_cap);
hipError_t scan_attributes(int np2, int np3, int gk, int *vgprs, int *lds_bytes);
hipError_t launch_merge(int n_tasks, hipStream_t st, const Task *tasks, Cand *parts, Cand *results);
hipError_t launch_finalize(int n_tasks, int max_k, hipStream_t st, const Task *tasks, const Cand *results,
                           const ResultLayout *layout, char *out);
hipError_t launch_init_counters(hipStream_t st, unsigned long long *queues, int nq, unsigned *cand_counts,
                                unsigned long long *thrs, int n_tasks, unsigned *hist);
// fn 0: genotype rows, 1: contingency tables (of combos), 2: MI (of tables)
hipError_t launch_function(int fn, int order, hipStream_t st, const DsView &d, const int32_t *combos,
                           const uint32_t *tables, unsigned long long n, void *out, int *err, int grid,
                           long long score_const);
hipError_t launch_reseed(int n_tasks, hipStream_t st, const Task *tasks, const Cand *results);
hipError_t launch_items(hipStream_t st, int kind, int M, int np, unsigned long long *out);
hipError_t launch_store(hipStream_t st, const void *src, size_t bytes, void *dst);
hipError_t launch_scatter(hipStream_t st, const char *block, int top_k, int order, int32_t *combos, float *scores,
                          uint32_t *tables, int32_t *n);
hipError_t launch_pack(hipStream_t st, const uint8_t *geno, long long ld, const int32_t *idx, const DsView &d,
                       v4u *masks, int *err);
hipError_t launch_classidx(hipStream_t st, const uint8_t *pheno, int N, int n_case, int32_t *idx, int *err);
hipError_t launch_singles(hipStream_t st, const DsView &d, uint32_t *single);
hipError_t launch_qpack(hipStream_t st, const DsView &d, v4u *qa, v4u *qb);
hipError_t launch_qpack8(hipStream_t st, const DsView &d, v4u *qa8, v4u *qb8);

// runtime helpers shared with the server
uint64_t binom_u64(int64_t n, int64_t k);
int get_items(Ctx *c, int variant, int M, int np, const void **d, unsigned long long *n);
int check_desc(Ctx *c, const epi_scan_desc &d, Dataset **out);
void pick_group_kernel(const std::vector<int> &orders, int np_hint, int *np2, int *np3, int *gk);
int group_of_order(int order, int np);
int size_bucket(const Dataset *d);
bool r4_fits(const Dataset *d);
int tuned_np_lookup(Ctx *c, int order, const Dataset *d);
bool seg_pinned(Ctx *c, int order, const Dataset *d);
int default_np3(Ctx *c, const Dataset *d);
bool np3_usable(const Dataset *d, int np);
int grid_for(Ctx *c, int np2, int np3, int gk, unsigned long long items, int tab_cap, int kmax, int stage_cap);
int stage_cap_for(int np2, int np3, int w4_max);
int tab_entries_for(const Dataset *d, int variant, int np, bool both);
void set_pair_form(Task &t, const Dataset *d, int order, int variant, int np);
int group_tab_cap(int np2, int np3, int gk, int cap_both, int cap_first, int kmax, int stage_cap);

Ctx *as_ctx(epi_ctx *c);
int key_bits_for(int order);
void load_tune_cache(Ctx *c);
// Device memory an allocation-free plan is carved from.
struct PlanArena {
    char *base;
    size_t cap;
};
int plan_build(Ctx *c, const epi_scan_desc *descs, int n, bool persistent, bool graph, Plan **out, int force_np,
               bool check = false, const PlanArena *arena = nullptr);
bool use_r4(Ctx *c, const Dataset *d);
uint64_t pair_table_bytes(int variant, int M);
uint64_t triple_table_bytes(int M);
int plan_run(Ctx *c, Plan *p, hipStream_t st, unsigned long long item_cap);
int plan_wait(Plan *p);
int plan_results(Plan *p, int index, int capacity, int32_t *combos, float *scores, uint32_t *tables,
                 int32_t *n_written);
int pack_error(int bits);
void plan_free(Ctx *c, Plan *p);
void server_shutdown_all(Ctx *c);

}  // namespace epi
