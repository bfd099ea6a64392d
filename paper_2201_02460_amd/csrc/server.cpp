// Serving: continuous batching of scan requests on resident datasets.
//
// A server thread runs launch rounds.  Each round it
//   1. admits queued requests (first come, first served) while the number of
//      active requests and the device bytes their buffers need stay within
//      the configured limits;
//   2. gives every active request a slice of its remaining work items, sized
//      so that a round is a few milliseconds of device work, and runs all the
//      slices in one persistent launch of the scan kernel (order-3 requests
//      run their pair sub-table pass in the round they are admitted);
//   3. compacts each request's candidates to its best K on the device, so the
//      next round adds to a short list;
//   4. finishes the requests whose work is done: result tables, scores and
//      combinations are copied to host memory and the request's device
//      buffers return to the pool, which admits waiting requests next round.
// Requests that arrive while rounds run join the next round, so their work
// shares launches with older requests.  Every combination is scored by the
// same kernel code as a plain scan, so a request's results do not depend on
// what else was in its rounds.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "runtime_internal.hpp"

namespace epi {

using Clock = std::chrono::steady_clock;

struct Request {
    int id = 0;
    epi_scan_desc desc{};
    Dataset *ds = nullptr;
    int state = 0;  // 0 queued, 1 admitted, 2 done, 3 failed
    int rc = EPI_OK;
    std::string err;
    Clock::time_point t_submit, t_done;
    int variant = 0, np = 0, slot = -1;
    const void *items = nullptr, *emit_items = nullptr, *t3_items = nullptr;
    unsigned long long n_items = 0, cursor = 0, emit_n = 0, t3_n = 0, n_combos = 0;
    bool emit_done = false;
    bool finishing = false;  // its last slice is in the round in flight (results not yet read)
    // pilot pass in the request's first round (matrix-core order 3, order 4
    // by reduced cells): items pilot_first .. + pilot_n - 1
    int pilot_n = 0;
    unsigned long long pilot_first = 0;
    bool big_tab = false;  // its screening table lowers the kernel's workgroups per CU
    void *pairs = nullptr, *triples = nullptr, *cand = nullptr;
    unsigned cand_cap = 0;
    uint64_t footprint = 0;
    std::vector<char> out;  // result block copied from the device
    bool holds_ds = false;  // counted in ds->users until the request is done or failed
};

// The request no longer reads its dataset (done or failed).
static void drop_dataset(Request *r) {
    if (r->holds_ds) r->ds->users.fetch_sub(1);
    r->holds_ds = false;
}

struct Server {
    Ctx *ctx = nullptr;
    int id = 0;
    epi_server_config cfg{};
    hipStream_t stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};  // end of the two rounds that may be in flight
    // side streams for a round's launch groups: each group's launch ends in a
    // tail (the waves that finish first wait for the last items), which the
    // next group, on another stream, fills
    static constexpr int kSide = 2;
    hipStream_t side[kSide] = {};
    hipEvent_t ev_fork = nullptr, ev_join[kSide] = {};
    std::thread thread;
    std::mutex mu;
    std::condition_variable cv;
    bool stopping = false;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<int, std::shared_ptr<Request>> all;
    std::vector<std::shared_ptr<Request>> active;
    std::vector<int> free_slots;
    int next_req = 1;
    uint64_t budget = 0, used = 0;
    int grid_max = 1;
    // device state: per-slot counters, per-round scratch
    void *d_counters = nullptr, *d_tasks = nullptr, *d_results = nullptr, *d_parts = nullptr, *d_layout = nullptr,
         *d_out = nullptr;
    // host staging of a round's task and layout arrays, one per round in
    // flight (a round's copies read them when the stream reaches them)
    void *h_tasks[2] = {nullptr, nullptr}, *h_out = nullptr, *h_layout[2] = {nullptr, nullptr};
    int buf = 0;  // staging buffer and event of the next round
    bool backlog = false;  // requests waiting for admission (server thread only)
    unsigned long long *d_queues = nullptr, *d_thr = nullptr;
    unsigned *d_hist = nullptr;  // kHistWords per slot
    unsigned *d_cand_count = nullptr;
    long long out_block = 0;
    int max_round_tasks = 0;
    // stats
    uint64_t n_done = 0, rounds = 0, work_done = 0, peak_bytes = 0, peak_active = 0;
    int fatal = EPI_OK;
};

// Device work of a round, in combos x individuals: about 8 ms with up to four
// active requests, so a new arrival joins within a few milliseconds; with
// more requests in flight each still gets a useful slice per round, up to
// eight times that.
static const double kRoundWork = 4e11;
// With rounds_in_flight = 0, a second round is enqueued behind the running one
// only while the next round's work stays below this (about 5 ms of the order-3
// kernel): the host's round gap then costs several per cent of the device
// time, while a request that arrives meanwhile waits at most that long more.
static const double kPipelineWork = 2 * kRoundWork;
static const int kQueues = 32;

// Launch group of a request within a round, one per kernel instantiation:
// orders 2 and 3 per prefix block (their work items are built for that
// block), and each higher order.
// Launch group of a request in a round: its kernel instantiation, and apart
// from the others of that kernel when its screening table would cost the
// launch workgroups per CU (the group's LDS table takes its largest dataset).
static int round_group(const Request *r) { return group_of_order(r->desc.order, r->np) + (r->big_tab ? 100 : 0); }

static void free_request_buffers(Server *S, Request *r) {
    S->ctx->alloc.release(r->pairs);
    S->ctx->alloc.release(r->triples);
    S->ctx->alloc.release(r->cand);
    r->pairs = r->triples = r->cand = nullptr;
    if (r->slot >= 0) S->free_slots.push_back(r->slot);
    r->slot = -1;
    S->used -= r->footprint;
}

static void fail_request(Server *S, Request *r, int rc, const char *msg) {
    r->rc = rc;
    r->err = msg;
    r->state = 3;
    r->t_done = Clock::now();
    free_request_buffers(S, r);
    drop_dataset(r);
}

// Footprint and buffers of a request being admitted.
static int admit(Server *S, Request *r) {
    Ctx *c = S->ctx;
    const int o = r->desc.order;
    r->n_combos = binom_u64(r->ds->M, o);
    if (o == 2) {
        r->variant = kF2;
        const int t = tuned_np_lookup(c, 2, r->ds);
        r->np = t > 0 && (t != kNpMfma || r->ds->qa) ? t : 4;
    } else if (o == 3) {
        r->variant = kF3;
        r->np = default_np3(c, r->ds);
    } else {
        r->variant = o == 4 && use_r4(c, r->ds) ? kR4 : kGeneric;
        r->np = kGenRanksHost;
        r->n_items = (r->n_combos + 64ull * kGenRanksHost - 1) / (64ull * kGenRanksHost);
    }
    const bool sub = o == 3 || r->variant == kR4;  // pair sub-table pass
    int rc;
    if ((r->variant == kF2 || r->variant == kF3) && (rc = get_items(c, r->variant, r->ds->M, r->np, &r->items, &r->n_items)))
        return rc;
    if (sub && (rc = get_items(c, kF2, r->ds->M, 4, &r->emit_items, &r->emit_n))) return rc;
    if (r->variant == kR4 && (rc = get_items(c, kF3, r->ds->M, kNpMfma, &r->t3_items, &r->t3_n))) return rc;
    r->cand_cap = (unsigned)((unsigned long long)S->grid_max * 4 * r->desc.top_k + r->desc.top_k + 64);
    r->pilot_n = pilot_items_for(r->variant, r->np, r->n_items, r->desc.top_k, r->ds->N, Plan::kTabMax,
                                 S->grid_max * 4);
    r->big_tab = table_lowers_occupancy(r->ds, r->variant, r->np, o, r->desc.top_k);
    r->pilot_first = (r->n_items - (unsigned long long)r->pilot_n) / 2;
    const uint64_t pair_bytes = sub ? pair_table_bytes(r->variant, r->ds->M) : 0;
    const uint64_t trip_bytes = r->variant == kR4 ? triple_table_bytes(r->ds->M) : 0;
    r->footprint = pair_bytes + trip_bytes + (uint64_t)r->cand_cap * sizeof(Cand);
    if (S->used + r->footprint > S->budget) return EPI_ENOMEM;
    auto undo = [&](int code) {
        c->alloc.release(r->pairs);
        c->alloc.release(r->triples);
        r->pairs = r->triples = nullptr;
        return code;
    };
    if (pair_bytes && (rc = c->alloc.alloc(pair_bytes, &r->pairs))) return undo(rc);
    if (trip_bytes && (rc = c->alloc.alloc(trip_bytes, &r->triples))) return undo(rc);
    if ((rc = c->alloc.alloc((size_t)r->cand_cap * sizeof(Cand), &r->cand))) return undo(rc);
    S->used += r->footprint;
    S->peak_bytes = std::max<uint64_t>(S->peak_bytes, S->used);
    r->slot = S->free_slots.back();
    S->free_slots.pop_back();
    r->state = 1;
    return EPI_OK;
}

static Task make_task(Server *S, Request *r) {
    Task t;
    memset(&t, 0, sizeof t);
    t.ds = r->ds->view;
    t.pairs = (uint32_t *)r->pairs;
    t.triples = (uint32_t *)r->triples;
    t.items = (const unsigned long long *)r->items;
    t.n_items = r->n_items;
    t.n_combos = r->n_combos;
    t.score_const = r->ds->score_const;
    t.cand = (Cand *)r->cand;
    t.cand_count = S->d_cand_count + r->slot;
    t.thr = S->d_thr + r->slot;
    t.hist = S->d_hist + (size_t)r->slot * kHistWords;
    t.cand_cap = r->cand_cap;
    t.variant = r->variant;
    t.order = r->desc.order;
    t.top_k = r->desc.top_k;
    t.np = r->np;
    t.key_bits = key_bits_for(r->desc.order);
    t.pilot_first = r->pilot_first;
    t.pilot_n = r->pilot_n;
    return t;
}

#define SRV_HIPCHK(x)                                                        \
    do {                                                                     \
        hipError_t e_ = (x);                                                 \
        if (e_ != hipSuccess) return fail(EPI_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

// combos x individuals of one work item of a request
static unsigned long long item_work(const Request *r) {
    return (unsigned long long)(r->variant == kGeneric ? 64 * kGenRanksHost : 64 * r->np) * r->ds->N;
}

// Each request's share of the next round's work: a round is kRoundWork split
// equally, growing up to 8x with more than four requests (so that one slice
// per request stays useful), and kBacklogRounds times that while requests
// wait for admission: rounds of small slices cost the scan kernels several
// per cent of their time, which only matters while the device is the
// bottleneck; otherwise short rounds let new requests start sooner.
static const double kBacklogRounds = 4;
static double round_share(const Server *S) {
    size_t live = 0;
    for (auto &r : S->active) live += r->finishing ? 0 : 1;
    const double na = (double)std::max<size_t>(1, live);
    return kRoundWork * std::min(8.0, std::max(1.0, na / 4.0)) * (S->backlog ? kBacklogRounds : 1.0) / na;
}

// Work items of a request's slice in the next round (its remaining items if
// they fit its share).
static unsigned long long slice_items(const Request *r, double share) {
    const unsigned long long n =
        (unsigned long long)std::max(1.0, share / (double)std::max<unsigned long long>(item_work(r), 1));
    return std::min(n, r->n_items - r->cursor);
}

// Each running request's slice of the next round, in work items.
static std::vector<std::pair<Request *, unsigned long long>> round_slices(const Server *S) {
    const double share = round_share(S);
    std::vector<std::pair<Request *, unsigned long long>> sl;
    for (auto &r : S->active)
        if (!r->finishing) sl.push_back({r.get(), slice_items(r.get(), share)});
    return sl;
}

// combos x individuals the next round would cover; -1 if no request is left
// to run (every active one is finishing in the round in flight).
static double next_round_work(const Server *S) {
    double w = -1;
    for (auto &p : round_slices(S)) w = std::max(w, 0.0) + (double)p.second * (double)item_work(p.first);
    return w;
}

// A round enqueued on the server stream: the requests it finishes and its
// event.  Two rounds may be in flight: the host builds and enqueues the next
// round while the device runs the current one, then reads the current one's
// results.
struct RoundDone {
    std::vector<Request *> fin;
    int ev = 0;
};

// Build and enqueue one round over the active requests that are not already
// finishing; returns EPI_OK or a device error (which stops the server).
static int run_round(Server *S, RoundDone *done) {
    Ctx *c = S->ctx;
    hipStream_t st = S->stream;
    // newly admitted requests: zero their counters
    for (auto &r : S->active)
        if (!r->finishing && !r->emit_done && r->cursor == 0) {
            SRV_HIPCHK(launch_init_counters(st, nullptr, 0, S->d_cand_count + r->slot, S->d_thr + r->slot, 1,
                                            S->d_hist + (size_t)r->slot * kHistWords));
        }
    // slices: finishing requests first (their merge results feed finalize)
    std::vector<std::pair<Request *, unsigned long long>> fin, cont;
    for (auto &p : round_slices(S)) (p.first->cursor + p.second >= p.first->n_items ? fin : cont).push_back(p);
    std::vector<std::pair<Request *, unsigned long long>> order = fin;
    order.insert(order.end(), cont.begin(), cont.end());
    const int nt = (int)order.size();
    // task array: [main tasks][emit tasks][launch-group copies]
    Task *ht = (Task *)S->h_tasks[S->buf];
    int ti = 0;
    for (auto &pr : order) ht[ti++] = make_task(S, pr.first);
    const int emit_off = ti;
    unsigned long long emit_total = 0;
    int emit_w4 = 1;
    for (auto &pr : order) {
        Request *r = pr.first;
        if ((r->desc.order != 3 && r->variant != kR4) || r->emit_done) continue;
        Task t = make_task(S, r);
        t.variant = kF2Emit;
        t.items = (const unsigned long long *)r->emit_items;
        t.n_items = r->emit_n;
        t.item_base = emit_total;
        t.np = 4;
        t.order = 2;
        set_pair_form(t, r->ds, r->desc.order, r->variant, r->np);
        emit_total += r->emit_n;
        emit_w4 = std::max(emit_w4, std::max(r->ds->w4[0], r->ds->w4[1]));
        ht[ti++] = t;
    }
    const int n_emit = ti - emit_off;
    // triplet sub-table passes of new reduced order-4 requests (matrix cores)
    const int t3_off = ti;
    unsigned long long t3_total = 0;
    for (auto &pr : order) {
        Request *r = pr.first;
        if (r->variant != kR4 || r->emit_done) continue;
        Task t = make_task(S, r);
        t.variant = kF3Emit;
        t.items = (const unsigned long long *)r->t3_items;
        t.n_items = r->t3_n;
        t.item_base = t3_total;
        t.np = kNpMfma;
        t.order = 3;
        t3_total += r->t3_n;
        ht[ti++] = t;
    }
    const int n_t3 = ti - t3_off;
    // launch groups by kernel instantiation
    struct G {
        int np2, np3, gk, off, n, tab_cap, kmax, stage;
        unsigned long long total;
        int pilot_off, pilot_tasks;  // the pilot launch's task copies (requests in their first round)
        unsigned long long pilot_total;
    };
    std::vector<G> groups;
    for (int key : {30 + kNpMfma, 30 + kNpMfma2, 30 + kNpMfmaI8, 38, 34, 32, 31, 20 + kNpMfma, 22, 24, 28, 4, 5,
                    130 + kNpMfma, 130 + kNpMfma2, 130 + kNpMfmaI8, 138, 134, 132, 131, 120 + kNpMfma, 122, 124, 128,
                    104, 105}) {
        std::vector<int> orders;
        G g{0, 0, 0, ti, 0, 0, 1, 0, 0, 0, 0, 0};
        int np_hint = 4;  // the group's prefix block: every request of a key has the same
        for (int i = 0; i < nt; ++i) {
            Request *r = order[i].first;
            if (round_group(r) != key) continue;
            orders.push_back(r->desc.order);
            np_hint = r->np;
        }
        if (orders.empty()) continue;
        pick_group_kernel(orders, np_hint, &g.np2, &g.np3, &g.gk);
        g.stage = stage_cap_for(g.np2, g.np3, 0);
        int cap_both = 0, cap_first = 0;
        std::vector<Request *> members;  // the group's requests, in copy order
        for (int i = 0; i < nt; ++i) {
            Request *r = order[i].first;
            if (round_group(r) != key) continue;
            members.push_back(r);
            Task t = ht[i];
            t.item_base = g.total;
            t.first_item = r->cursor;
            g.total += order[i].second;
            ht[ti++] = t;
            g.n++;
            g.kmax = std::max(g.kmax, r->desc.top_k);
            g.stage = std::max(g.stage, stage_cap_for(g.np2, g.np3, std::max(r->ds->w4[0], r->ds->w4[1])));
            cap_both = std::max(cap_both, tab_entries_for(r->ds, r->variant, r->np, true));
            cap_first = std::max(cap_first, tab_entries_for(r->ds, r->variant, r->np, false));
        }
        g.tab_cap = group_tab_cap(g.np2, g.np3, g.gk, cap_both, cap_first, g.kmax, g.stage);
        g.kmax = group_list_cap(g.np2, g.np3, g.gk, g.tab_cap, g.kmax, g.stage);
        // requests in their first round with a pilot pass: copies numbered
        // in the pilot launch
        g.pilot_off = ti;
        for (int k = 0; k < g.n; ++k) {
            Request *r = members[k];
            if (r->cursor != 0 || r->pilot_n == 0) continue;
            if (ti >= S->max_round_tasks) return fail(EPI_EDEVICE, "server round task array overflow");
            Task t = ht[g.off + k];
            t.pilot_base = g.pilot_total;
            g.pilot_total += (unsigned long long)r->pilot_n;
            ht[ti++] = t;
            g.pilot_tasks++;
        }
        groups.push_back(g);
    }
    if (ti > S->max_round_tasks) return fail(EPI_EDEVICE, "server round task array overflow");
    SRV_HIPCHK(hipMemcpyAsync(S->d_tasks, ht, (size_t)ti * sizeof(Task), hipMemcpyHostToDevice, st));
    const Task *dt = (const Task *)S->d_tasks;
    const int nq = 2 + (int)groups.size();
    if (nq > kQueues) return fail(EPI_EDEVICE, "server round has too many launch groups");
    SRV_HIPCHK(launch_init_counters(st, S->d_queues, nq, nullptr, nullptr, 0, nullptr));
    if (n_emit > 0) {
        const int es = stage_cap_for(4, 0, emit_w4);
        const int eg = grid_for(c, 4, 0, 0, emit_total, 0, 1, es);
        SRV_HIPCHK(launch_scan(4, 0, 0, eg, st, dt + emit_off, n_emit, emit_total, S->d_queues, c->d_binom,
                               c->bstride, 0, 1, es));
    }
    if (n_t3 > 0) {
        const int ts = stage_cap_for(0, kNpMfma, 0);
        const int tg = grid_for(c, 0, kNpMfma, 0, t3_total, 0, 1, ts);
        SRV_HIPCHK(launch_scan(0, kNpMfma, 0, tg, st, dt + t3_off, n_t3, t3_total, S->d_queues + 1, c->d_binom,
                               c->bstride, 0, 1, ts));
    }
    // launch groups round-robin over the server stream and the side streams
    // (they touch disjoint requests and queue counters; the side streams
    // start after the pair passes above and the merge below waits for them)
    const int n_side = std::min<int>(Server::kSide, (int)groups.size() - 1);
    if (n_side > 0) {
        SRV_HIPCHK(hipEventRecord(S->ev_fork, st));
        for (int k = 0; k < n_side; ++k) SRV_HIPCHK(hipStreamWaitEvent(S->side[k], S->ev_fork, 0));
    }
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const G &g = groups[gi];
        const int lane_s = (int)(gi % (size_t)(Server::kSide + 1));
        hipStream_t gs = lane_s == 0 ? st : S->side[lane_s - 1];
        const int grid = grid_for(c, g.np2, g.np3, g.gk, g.total, g.tab_cap, g.kmax, g.stage);
        if (g.pilot_total > 0)
            SRV_HIPCHK(launch_pilot(g.np2, g.np3, g.gk,
                                    (int)std::min<unsigned long long>(std::min(grid, S->grid_max), g.pilot_total / 4),
                                    gs, dt + g.pilot_off, g.pilot_tasks, g.pilot_total, c->d_binom, c->bstride,
                                    g.tab_cap, g.kmax, g.stage));
        SRV_HIPCHK(launch_scan(g.np2, g.np3, g.gk, std::min(grid, S->grid_max), gs, dt + g.off, g.n, g.total,
                               S->d_queues + 2 + gi, c->d_binom, c->bstride, g.tab_cap, g.kmax, g.stage));
    }
    for (int k = 0; k < n_side; ++k) {
        SRV_HIPCHK(hipEventRecord(S->ev_join[k], S->side[k]));
        SRV_HIPCHK(hipStreamWaitEvent(st, S->ev_join[k], 0));
    }
    // compact every request's candidates to its best K; finish the done ones
    SRV_HIPCHK(launch_merge(nt, st, dt, (Cand *)S->d_parts, (Cand *)S->d_results));
    SRV_HIPCHK(launch_reseed(nt, st, dt, (const Cand *)S->d_results));
    if (!fin.empty()) {
        ResultLayout *hl = (ResultLayout *)S->h_layout[S->buf];
        int maxk = 1;
        for (size_t i = 0; i < fin.size(); ++i) {
            Request *r = fin[i].first;
            hl[i].offset = (long long)r->slot * S->out_block;
            hl[i].top_k = r->desc.top_k;
            hl[i].order = r->desc.order;
            maxk = std::max(maxk, r->desc.top_k);
        }
        SRV_HIPCHK(hipMemcpyAsync(S->d_layout, hl, fin.size() * sizeof(ResultLayout), hipMemcpyHostToDevice, st));
        SRV_HIPCHK(launch_finalize((int)fin.size(), maxk, st, dt, (const Cand *)S->d_results,
                                   (const ResultLayout *)S->d_layout, (char *)S->d_out));
        for (auto &pr : fin) {
            Request *r = pr.first;
            const long long off = (long long)r->slot * S->out_block;
            SRV_HIPCHK(hipMemcpyAsync((char *)S->h_out + off, (char *)S->d_out + off,
                                      (size_t)result_block_bytes(r->desc.top_k, r->desc.order), hipMemcpyDeviceToHost,
                                      st));
        }
    }
    SRV_HIPCHK(hipEventRecord(S->ev[S->buf], st));
    done->ev = S->buf;
    S->buf ^= 1;
    // bookkeeping of what was enqueued: the next round takes the following
    // items, and the finishing requests sit out until their results are read
    std::lock_guard<std::mutex> g(S->mu);
    S->rounds++;
    for (auto &pr : order) {
        Request *r = pr.first;
        // combinations covered so far, estimated as items x the combinations
        // of a full item up to the request's total, and the total once its
        // last item is in
        const unsigned long long per = item_work(r) / (unsigned long long)r->ds->N;
        auto covered = [&] {
            return r->cursor >= r->n_items ? r->n_combos : std::min<unsigned long long>(r->cursor * per, r->n_combos);
        };
        const unsigned long long before = covered();
        r->cursor += pr.second;
        r->emit_done = true;
        const unsigned long long after = covered();
        S->work_done += (after - before) * (unsigned long long)r->ds->N;
    }
    done->fin.clear();
    for (auto &pr : fin) {
        pr.first->finishing = true;
        done->fin.push_back(pr.first);
    }
    return EPI_OK;
}

// Wait for an enqueued round and hand its finishing requests their results.
static int complete_round(Server *S, const RoundDone &done) {
    SRV_HIPCHK(hipEventSynchronize(S->ev[done.ev]));
    std::lock_guard<std::mutex> g(S->mu);
    for (Request *r : done.fin) {
        const long long off = (long long)r->slot * S->out_block;
        const long long bytes = result_block_bytes(r->desc.top_k, r->desc.order);
        r->out.assign((char *)S->h_out + off, (char *)S->h_out + off + bytes);
        r->state = 2;
        r->t_done = Clock::now();
        r->finishing = false;
        free_request_buffers(S, r);
        drop_dataset(r);
        S->n_done++;
    }
    S->active.erase(std::remove_if(S->active.begin(), S->active.end(),
                                   [](const std::shared_ptr<Request> &r) { return r->state != 1; }),
                    S->active.end());
    return EPI_OK;
}

static void server_main(Server *S) {
    (void)hipSetDevice(S->ctx->device);
    RoundDone pending;
    bool have_pending = false;
    for (;;) {
        double work = -1;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait_for(lk, std::chrono::milliseconds(50),
                           [&] { return S->stopping || !S->queue.empty() || !S->active.empty(); });
            // admission: first come, first served, by slots and device bytes
            while (!S->queue.empty() && (int)S->active.size() < S->cfg.max_active && !S->free_slots.empty()) {
                auto r = S->queue.front();
                const int rc = admit(S, r.get());
                if (rc == EPI_ENOMEM && !S->active.empty()) break;  // wait for memory to free up
                S->queue.pop_front();
                if (rc != EPI_OK) {
                    r->rc = rc;
                    r->err = last_error();
                    r->state = 3;
                    r->t_done = Clock::now();
                    drop_dataset(r.get());
                    continue;
                }
                S->active.push_back(r);
            }
            S->peak_active = std::max<uint64_t>(S->peak_active, S->active.size());
            S->backlog = !S->queue.empty();
            if (S->active.empty()) {
                if (S->stopping && S->queue.empty()) return;
                continue;
            }
            work = next_round_work(S);
        }
        const int depth = S->cfg.rounds_in_flight;
        const bool overlap = work >= 0 && (depth == 2 || (depth == 0 && work <= kPipelineWork));
        int rc = EPI_OK;
        if (have_pending && !overlap) {
            // read the round in flight first; requests that arrive meanwhile
            // then join the next round
            rc = complete_round(S, pending);
            have_pending = false;
            if (rc == EPI_OK) continue;
        } else if (work >= 0) {
            // enqueue the next round, then read the one before it
            RoundDone next;
            rc = run_round(S, &next);
            if (rc == EPI_OK && have_pending) rc = complete_round(S, pending);
            have_pending = rc == EPI_OK;
            pending = next;
        }
        if (rc != EPI_OK) {
            // no round in flight past this point
            (void)hipStreamSynchronize(S->stream);
            for (int k = 0; k < Server::kSide; ++k) (void)hipStreamSynchronize(S->side[k]);
            std::lock_guard<std::mutex> g(S->mu);
            S->fatal = rc;
            for (auto &r : S->active) fail_request(S, r.get(), rc, "device error in a serving round");
            S->active.clear();
            for (auto &r : S->queue) {
                r->rc = rc;
                r->state = 3;
                drop_dataset(r.get());
            }
            S->queue.clear();
            return;
        }
    }
}

static void server_free(Server *S) {
    Ctx *c = S->ctx;
    c->alloc.release(S->d_counters);
    c->alloc.release(S->d_tasks);
    c->alloc.release(S->d_results);
    c->alloc.release(S->d_parts);
    c->alloc.release(S->d_layout);
    c->alloc.release(S->d_out);
    for (int b = 0; b < 2; ++b) {
        if (S->h_tasks[b]) (void)hipHostFree(S->h_tasks[b]);
        if (S->h_layout[b]) (void)hipHostFree(S->h_layout[b]);
        if (S->ev[b]) (void)hipEventDestroy(S->ev[b]);
    }
    if (S->h_out) (void)hipHostFree(S->h_out);
    for (int k = 0; k < Server::kSide; ++k) {
        if (S->side[k]) (void)hipStreamDestroy(S->side[k]);
        if (S->ev_join[k]) (void)hipEventDestroy(S->ev_join[k]);
    }
    if (S->ev_fork) (void)hipEventDestroy(S->ev_fork);
    if (S->stream) (void)hipStreamDestroy(S->stream);
}

static void server_join(Server *S) {
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stopping = true;
    }
    S->cv.notify_all();
    if (S->thread.joinable()) S->thread.join();
}

void server_shutdown_all(Ctx *c) {
    for (auto &kv : c->servers) {
        server_join(kv.second.get());
        server_free(kv.second.get());
    }
    c->servers.clear();
}

static Server *server_of(Ctx *C, int32_t id) {
    std::lock_guard<std::mutex> g(C->mu);
    auto it = C->servers.find(id);
    return it == C->servers.end() ? nullptr : it->second.get();
}

}  // namespace epi

using namespace epi;

#define CTX_OR_FAIL(ctx)                                                  \
    if (!(ctx)) return fail(EPI_EINVAL, "null context");                  \
    Ctx *C = as_ctx(ctx);                                                 \
    if (hipSetDevice(C->device) != hipSuccess) return fail(EPI_EDEVICE, "hipSetDevice failed");

#define HIPCHK(x)                                                                        \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) return fail(EPI_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

extern "C" {

int epi_server_start(epi_ctx *ctx, const epi_server_config *cfg, int32_t *server_id) {
    clear_error();
    CTX_OR_FAIL(ctx);
    if (!cfg || !server_id || cfg->max_active < 1 || cfg->max_active > 4096 || cfg->rounds_in_flight < 0 ||
        cfg->rounds_in_flight > 2)
        return fail(EPI_EINVAL, "bad server configuration");
    auto S = std::make_shared<Server>();
    S->ctx = C;
    S->cfg = *cfg;
    S->budget = cfg->request_budget ? cfg->request_budget : C->alloc.budget;
    // the largest persistent grid any round may launch (in 4-wave workgroups)
    static const int kRoundKernels[][3] = {{2, 0, 0}, {4, 0, 0}, {8, 0, 0}, {0, 1, 0}, {0, 2, 0}, {0, 4, 0},
                                           {0, 8, 0}, {0, kNpMfma, 0}, {0, kNpMfma2, 0}, {0, kNpMfmaI8, 0},
                                           {0, 0, 4}, {0, 0, 5}, {kNpMfma, 0, 0}};
    S->grid_max = 1;
    for (const auto &k : kRoundKernels)
        S->grid_max = std::max(S->grid_max,
                               grid_for(C, k[0], k[1], k[2], ~0ull >> 8, 0, 1, stage_cap_for(k[0], k[1], 1)));
    const int A = cfg->max_active;
    S->max_round_tasks = 5 * A + 4;  // main, pair passes, triplet passes, group copies, pilot copies
    S->out_block = result_block_bytes(EPI_MAX_TOP_K, EPI_SERVE_MAX_ORDER);
    int rc;
    auto cleanup = [&](int code) {
        server_free(S.get());
        return code;
    };
    // queue counters: one for the pair pass and one per launch group (at most
    // eight groups: order 2, order 3 per prefix block, orders 4 and 5)
    if ((rc = C->alloc.alloc((size_t)kQueues * 8 + (size_t)A * 8 + (size_t)A * 4 + (size_t)A * kHistWords * 4,
                             &S->d_counters)))
        return cleanup(rc);
    S->d_queues = (unsigned long long *)S->d_counters;
    S->d_thr = S->d_queues + kQueues;
    S->d_cand_count = (unsigned *)(S->d_thr + A);
    S->d_hist = S->d_cand_count + A;
    if ((rc = C->alloc.alloc((size_t)S->max_round_tasks * sizeof(Task), &S->d_tasks))) return cleanup(rc);
    if ((rc = C->alloc.alloc((size_t)A * kMaxTopK * sizeof(Cand), &S->d_results))) return cleanup(rc);
    if ((rc = C->alloc.alloc((size_t)A * kMergeParts * kMaxTopK * sizeof(Cand), &S->d_parts))) return cleanup(rc);
    if ((rc = C->alloc.alloc((size_t)A * sizeof(ResultLayout), &S->d_layout))) return cleanup(rc);
    if ((rc = C->alloc.alloc((size_t)A * S->out_block, &S->d_out))) return cleanup(rc);
    for (int b = 0; b < 2; ++b) {
        HIPCHK(hipHostMalloc(&S->h_tasks[b], (size_t)S->max_round_tasks * sizeof(Task), hipHostMallocDefault));
        HIPCHK(hipHostMalloc(&S->h_layout[b], (size_t)A * sizeof(ResultLayout), hipHostMallocDefault));
        HIPCHK(hipEventCreateWithFlags(&S->ev[b], hipEventDisableTiming));
    }
    HIPCHK(hipHostMalloc(&S->h_out, (size_t)A * S->out_block, hipHostMallocDefault));
    HIPCHK(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
    for (int k = 0; k < Server::kSide; ++k) {
        HIPCHK(hipStreamCreateWithFlags(&S->side[k], hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&S->ev_join[k], hipEventDisableTiming));
    }
    HIPCHK(hipEventCreateWithFlags(&S->ev_fork, hipEventDisableTiming));
    for (int i = A - 1; i >= 0; --i) S->free_slots.push_back(i);
    {
        std::lock_guard<std::mutex> g(C->mu);
        S->id = C->next_id++;
        C->servers[S->id] = S;
    }
    S->thread = std::thread(server_main, S.get());
    *server_id = S->id;
    return EPI_OK;
}

int epi_server_submit(epi_ctx *ctx, int32_t server_id, int32_t dataset_id, int32_t order, int32_t top_k,
                      int32_t *request_id) {
    clear_error();
    CTX_OR_FAIL(ctx);
    Server *S = server_of(C, server_id);
    if (!S) return fail(EPI_ENOTFOUND, "unknown server %d", server_id);
    if (!request_id) return fail(EPI_EINVAL, "null request_id");
    epi_scan_desc d{dataset_id, order, top_k, 0};
    Dataset *ds = nullptr;
    {
        std::lock_guard<std::mutex> g(C->mu);
        int rc = check_desc(C, d, &ds);
        if (rc == EPI_OK && order > EPI_SERVE_MAX_ORDER)
            rc = fail(EPI_EUNSUPPORTED, "order %d > %d for served requests", order, EPI_SERVE_MAX_ORDER);
        if (rc) return rc;
        // counted while the context lock is held, so epi_unload either sees
        // the request or has already removed the dataset
        ds->users.fetch_add(1);
    }
    auto r = std::make_shared<Request>();
    r->desc = d;
    r->ds = ds;
    r->holds_ds = true;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> g(S->mu);
        if (S->stopping || S->fatal) {
            drop_dataset(r.get());
            if (S->stopping) return fail(EPI_EINVAL, "server is stopping");
            return fail(S->fatal, "server stopped after a device error");
        }
        r->id = S->next_req++;
        S->all[r->id] = r;
        S->queue.push_back(r);
    }
    S->cv.notify_all();
    *request_id = r->id;
    return EPI_OK;
}

int epi_server_poll(epi_ctx *ctx, int32_t server_id, int32_t request_id, int32_t *state) {
    clear_error();
    CTX_OR_FAIL(ctx);
    Server *S = server_of(C, server_id);
    if (!S) return fail(EPI_ENOTFOUND, "unknown server %d", server_id);
    if (!state) return fail(EPI_EINVAL, "null state");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->all.find(request_id);
    if (it == S->all.end()) return fail(EPI_ENOTFOUND, "unknown request %d", request_id);
    if (it->second->state == 3) return fail(it->second->rc, "request failed: %s", it->second->err.c_str());
    *state = it->second->state;
    return EPI_OK;
}

int epi_server_results(epi_ctx *ctx, int32_t server_id, int32_t request_id, int32_t capacity, int32_t *combos,
                       float *scores, uint32_t *tables, int32_t *n_written, double *latency_ms) {
    clear_error();
    CTX_OR_FAIL(ctx);
    Server *S = server_of(C, server_id);
    if (!S) return fail(EPI_ENOTFOUND, "unknown server %d", server_id);
    if (!n_written || capacity < 0) return fail(EPI_EINVAL, "bad arguments");
    std::shared_ptr<Request> r;
    {
        std::lock_guard<std::mutex> g(S->mu);
        auto it = S->all.find(request_id);
        if (it == S->all.end()) return fail(EPI_ENOTFOUND, "unknown request %d", request_id);
        r = it->second;
        if (r->state == 3) {
            S->all.erase(it);
            return fail(r->rc, "request failed: %s", r->err.c_str());
        }
        if (r->state != 2) return fail(EPI_ENOTREADY, "request %d not finished", request_id);
        S->all.erase(it);
    }
    const int K = r->desc.top_k, k = r->desc.order, cells = pow3i(k);
    const char *blk = r->out.data();
    const int32_t nv = *(const int32_t *)blk;
    if (((const int32_t *)blk)[1]) return pack_error(((const int32_t *)blk)[1]);
    const int32_t *hc = (const int32_t *)(blk + 16);
    const float *hs = (const float *)(blk + 16 + (size_t)K * k * 4);
    const uint32_t *ht = (const uint32_t *)(blk + 16 + (size_t)K * k * 4 + (size_t)K * 4);
    const int n = std::min(capacity, nv);
    if (n > 0 && (!combos || !scores)) return fail(EPI_EINVAL, "null combos/scores buffer");
    for (int i = 0; i < n; ++i) {
        memcpy(combos + (size_t)i * k, hc + (size_t)i * k, (size_t)k * 4);
        scores[i] = hs[i];
        if (tables) memcpy(tables + (size_t)i * 2 * cells, ht + (size_t)i * 2 * cells, (size_t)2 * cells * 4);
    }
    *n_written = n;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    return EPI_OK;
}

int epi_server_stats(epi_ctx *ctx, int32_t server_id, uint64_t out[5]) {
    clear_error();
    CTX_OR_FAIL(ctx);
    Server *S = server_of(C, server_id);
    if (!S) return fail(EPI_ENOTFOUND, "unknown server %d", server_id);
    if (!out) return fail(EPI_EINVAL, "null out");
    std::lock_guard<std::mutex> g(S->mu);
    out[0] = S->n_done;
    out[1] = S->rounds;
    out[2] = S->work_done;
    out[3] = S->peak_bytes;
    out[4] = S->peak_active;
    return EPI_OK;
}

int epi_server_stop(epi_ctx *ctx, int32_t server_id) {
    clear_error();
    CTX_OR_FAIL(ctx);
    std::shared_ptr<Server> S;
    {
        std::lock_guard<std::mutex> g(C->mu);
        auto it = C->servers.find(server_id);
        if (it == C->servers.end()) return fail(EPI_ENOTFOUND, "unknown server %d", server_id);
        S = it->second;
        C->servers.erase(it);
    }
    server_join(S.get());
    const int fatal = S->fatal;
    server_free(S.get());
    if (fatal) return fail(fatal, "server stopped after a device error");
    return EPI_OK;
}

}  // extern "C"
