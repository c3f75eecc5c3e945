// Serving loop: queued screening requests, admission by device-memory
// footprint, an LRU cache of resident reference tables, and merged batched
// launches per reference on a few lanes (one context + one stream each).
//
// The paper screens one reference against one template (Algorithm 1); this
// layer only schedules that screen for many requests.  Every request's
// result comes from the same kernels as oss_screen_batched: its templates
// take part in one batched star pass (possibly with other requests'
// templates on the same reference) and its own compaction writes its own
// mask and list, so the result does not depend on what it was merged with.
#include "api_internal.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <ctime>
#include <deque>
#include <map>
#include <new>
#include <thread>

using namespace oss;

namespace {

int64_t now_ns()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

enum ReqState { RQ_QUEUED, RQ_RUNNING, RQ_DONE, RQ_FAILED };

struct Req {
    int64_t id = 0;
    oss_request r{};
    std::vector<oss_template_feat> tmpl;
    std::vector<oss_probe> probes;
    int32_t need_r = 0;  // largest probe radius
    int state = RQ_QUEUED;
    int status = OSS_E_STATE;
    int64_t t_arr = 0, t_launch = 0, t_done = 0;
    void *out = nullptr;  // mask | list | count, one block
    size_t out_bytes = 0;  // bytes the outputs need
    size_t blk_bytes = 0;  // bytes of the block holding them (>= out_bytes)
    int slot = -1;        // pinned count slot while running
    int64_t count = 0;
    int batch = 0, hit = 0, lane = -1;
    uint64_t res_key = 0;

    int64_t hw() const { return (int64_t)r.desc.H * r.desc.W; }
    size_t mask_bytes() const { return (size_t)r.n_tmpl * (size_t)hw(); }
    uint8_t *mask() const { return static_cast<uint8_t *>(out); }
    oss_candidate *list() const
    {
        return reinterpret_cast<oss_candidate *>(static_cast<char *>(out) + align256(mask_bytes()));
    }
    int64_t *dcount() const
    {
        return reinterpret_cast<int64_t *>(static_cast<char *>(out) + align256(mask_bytes()) +
                                           align256((size_t)r.list_cap * sizeof(oss_candidate)));
    }
};

size_t output_bytes(const oss_request &r)
{
    return align256((size_t)r.n_tmpl * r.desc.H * r.desc.W) +
           align256((size_t)r.list_cap * sizeof(oss_candidate)) + 256;
}

// a lane's screen workspace for n_tmpl templates of H x W: the emission
// workspace, and scale-bit words when a group's radii span several passes
size_t workspace_bytes(int64_t n_tmpl, int H, int W, bool carry)
{
    return emit_workspace_bytes(n_tmpl, H, W) +
           (carry ? (size_t)n_tmpl * H * W * sizeof(uint32_t) : 0);
}

struct Resident {
    uint64_t key = 0;
    oss_ref *ref = nullptr;
    int users = 0;  // running lanes using it
    uint64_t lru = 0;
    hipEvent_t ready = nullptr;  // recorded after the build
};

struct Lane {
    oss_ctx *ctx = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Req *> reqs;
    uint64_t key = 0;
};

struct FreeBlock {
    size_t bytes;
    void *p;
};

bool same_desc(const oss_image_desc &a, const oss_image_desc &b)
{
    return a.H == b.H && a.W == b.W && a.dtype == b.dtype && a.bit_depth == b.bit_depth &&
           a.pitch_bytes == b.pitch_bytes;
}

constexpr int COUNT_SLOTS = 4096;
constexpr size_t PLAN_RESERVE = (size_t)1 << 20;  // plan bytes per slot, reserved at create

}  // namespace

struct oss_server {
    int device = 0;
    oss_server_config cfg{};
    std::vector<Lane> lanes;
    std::map<int64_t, Req *> reqs;
    std::deque<Req *> queue;
    std::vector<Resident> res;
    std::vector<FreeBlock> cache;  // released output blocks kept for reuse
    int64_t next_id = 1;
    uint64_t tick = 0;
    int64_t *counts = nullptr;  // pinned, COUNT_SLOTS entries
    std::vector<int> free_slots;
    size_t in_use = 0, peak = 0;
    oss_server_stats st{};

    size_t lane_ws(const Lane &l) const { return l.ctx->bits_cap + l.ctx->ews_cap; }
    void account(ptrdiff_t d)
    {
        in_use = (size_t)((ptrdiff_t)in_use + d);
        peak = std::max(peak, in_use);
    }
};

namespace {

Resident *find_res(oss_server *s, uint64_t key)
{
    for (Resident &r : s->res)
        if (r.key == key)
            return &r;
    return nullptr;
}

void drop_res(oss_server *s, Resident *r)
{
    const size_t bytes = r->ref->bytes;
    if (r->ready)
        (void)hipEventDestroy(r->ready);
    (void)oss_ref_release(r->ref);
    s->account(-(ptrdiff_t)bytes);
    s->st.evictions++;
    s->res.erase(s->res.begin() + (r - s->res.data()));
}

// Output blocks, evicted tables and idle lanes' workspaces are allocated
// and freed in stream order (on the lane that schedules), so admission never
// waits for the whole device.
void *alloc_out(oss_server *s, size_t bytes, size_t *got, hipStream_t st)
{
    // smallest cached block that is large enough and not more than twice the need
    int best = -1;
    for (int i = 0; i < (int)s->cache.size(); ++i)
        if (s->cache[i].bytes >= bytes && s->cache[i].bytes <= 2 * bytes &&
            (best < 0 || s->cache[i].bytes < s->cache[best].bytes))
            best = i;
    if (best >= 0) {
        void *p = s->cache[best].p;
        *got = s->cache[best].bytes;
        s->cache.erase(s->cache.begin() + best);
        return p;
    }
    void *p = nullptr;
    if (hipMallocAsync(&p, bytes, st) != hipSuccess)
        return nullptr;
    s->account((ptrdiff_t)bytes);
    *got = bytes;
    return p;
}

void free_cache(oss_server *s, hipStream_t st)
{
    for (FreeBlock &b : s->cache) {
        (void)hipFreeAsync(b.p, st);
        s->account(-(ptrdiff_t)b.bytes);
    }
    s->cache.clear();
}

// Free memory until `need` more bytes fit the budget: cached output blocks,
// then idle resident references (least recently used first, never `keep`),
// then idle lanes' workspaces (never `lane`).
bool make_room(oss_server *s, size_t need, uint64_t keep, bool keep_valid, int lane)
{
    const size_t budget = (size_t)s->cfg.memory_budget;
    if (s->in_use + need <= budget)
        return true;
    free_cache(s, s->lanes[lane].st);
    while (s->in_use + need > budget) {
        Resident *victim = nullptr;
        for (Resident &r : s->res)
            if (r.users == 0 && !(keep_valid && r.key == keep) && (!victim || r.lru < victim->lru))
                victim = &r;
        if (!victim)
            break;
        drop_res(s, victim);
    }
    for (int i = 0; i < (int)s->lanes.size() && s->in_use + need > budget; ++i) {
        Lane &l = s->lanes[i];
        if (i == lane || l.busy)
            continue;
        const size_t b = s->lane_ws(l);
        if (l.ctx->bits)
            (void)hipFreeAsync(l.ctx->bits, l.st);
        if (l.ctx->ews)
            (void)hipFreeAsync(l.ctx->ews, l.st);
        l.ctx->bits = nullptr;
        l.ctx->ews = nullptr;
        l.ctx->bits_cap = l.ctx->ews_cap = 0;
        s->account(-(ptrdiff_t)b);
    }
    return s->in_use + need <= budget;
}

void fail(oss_server *s, Req *q, int status)
{
    q->state = RQ_FAILED;
    q->status = status;
    q->t_done = now_ns();
    s->st.failed++;
}

// Retire finished lanes; returns the number of requests completed.
int retire(oss_server *s)
{
    int n = 0;
    for (Lane &l : s->lanes) {
        if (!l.busy)
            continue;
        const hipError_t e = hipEventQuery(l.done);
        if (e == hipErrorNotReady)
            continue;
        const int64_t t = now_ns();
        for (Req *q : l.reqs) {
            if (e == hipSuccess) {
                q->count = s->counts[q->slot];
                q->state = RQ_DONE;
                q->status = OSS_OK;
                q->t_done = t;
                s->st.completed++;
            } else {
                fail(s, q, OSS_E_DEVICE);
            }
            s->free_slots.push_back(q->slot);
            q->slot = -1;
            ++n;
        }
        if (Resident *r = find_res(s, l.key))
            r->users--;
        l.reqs.clear();
        l.busy = false;
    }
    return n;
}

// Launch `batch` (all on one reference) on lane `li`.
int launch(oss_server *s, int li, std::vector<Req *> &batch, Resident *r, bool hit)
{
    Lane &l = s->lanes[li];
    const Req *h = batch[0];
    const int64_t hw = h->hw();
    int T = 0;
    for (Req *q : batch)
        T += q->r.n_tmpl;
    std::vector<oss_template_feat> tm;
    std::vector<oss_tolerance> tols;
    std::vector<uint32_t> fms;
    std::vector<oss_probe> pr;
    int t0 = 0;
    for (Req *q : batch) {
        for (const oss_template_feat &f : q->tmpl) {
            tm.push_back(f);
            tols.push_back(q->r.tol);
            fms.push_back(q->r.feat_mask);
        }
        for (oss_probe p : q->probes) {
            p.template_id += t0;
            pr.push_back(p);
        }
        t0 += q->r.n_tmpl;
    }
    BatchHostPlan bp;
    int rc = make_batch_plan(r->ref, tm.data(), T, pr.data(), (int32_t)pr.size(), tols.data(),
                             fms.data(), l.ctx->batch_bucket, bp);
    if (rc != OSS_OK)
        return rc;
    const BuildGeom &g = r->ref->geom;
    const int strip = l.ctx->star_strip;
    const size_t ws0 = s->lane_ws(l);
    rc = screen_workspace(l.ctx, T, g.H, g.W, plan_carries(bp));
    s->account((ptrdiff_t)s->lane_ws(l) - (ptrdiff_t)ws0);
    if (rc != OSS_OK)
        return rc;
    if (!hit) {
        rc = oss_ref_build(r->ref, h->r.dev_pixels, l.st);
        if (rc != OSS_OK)
            return rc;
        if (hipEventRecord(r->ready, l.st) != hipSuccess)
            return OSS_E_DEVICE;
    } else if (hipStreamWaitEvent(l.st, r->ready, 0) != hipSuccess) {
        return OSS_E_DEVICE;
    }
    // each merged template's mask goes straight to its request's output
    std::vector<uint8_t *> masks;
    for (Req *q : batch)
        for (int t = 0; t < q->r.n_tmpl; ++t)
            masks.push_back(q->mask() + (int64_t)t * hw);
    PlanSlot *slot = nullptr;
    rc = batch_star(l.ctx, r->ref, bp, strip, l.ctx->star_blocks_per_xcd, masks.data(), l.st,
                    &slot);
    if (rc != OSS_OK)
        return rc;
    void *scan_ws = nullptr;
    const EmitOut eo = emit_out(l.ctx, T, g.H, g.W, &scan_ws);
    const int64_t segs_t = (int64_t)g.H * eo.n_chunks;
    t0 = 0;
    for (Req *q : batch) {
        // the request's own templates' segments, into its own list and count
        if (launch_list(eo.seg_count + segs_t * t0, eo.stage + segs_t * SEG_W * t0, q->r.n_tmpl,
                        g.H, g.W, q->list(), q->r.list_cap, q->dcount(), scan_ws, l.st,
                        &l.ctx->prof) != hipSuccess)
            return OSS_E_DEVICE;
        if (hipMemcpyAsync(s->counts + q->slot, q->dcount(), sizeof(int64_t),
                           hipMemcpyDeviceToHost, l.st) != hipSuccess)
            return OSS_E_DEVICE;
        t0 += q->r.n_tmpl;
    }
    if (hipEventRecord(slot->ev, l.st) != hipSuccess)
        return OSS_E_DEVICE;
    slot->used = true;
    if (hipEventRecord(l.done, l.st) != hipSuccess)
        return OSS_E_DEVICE;
    return OSS_OK;
}

// Completed requests whose outputs the caller has not released yet.
bool holds_results(const oss_server *s)
{
    for (const auto &kv : s->reqs)
        if ((kv.second->state == RQ_DONE || kv.second->state == RQ_FAILED) && kv.second->out)
            return true;
    return false;
}

bool any_busy(const oss_server *s)
{
    for (const Lane &l : s->lanes)
        if (l.busy)
            return true;
    return false;
}

// Queued requests that waited longer than the server's queue timeout fail.
void expire(oss_server *s)
{
    if (s->cfg.queue_timeout_ns <= 0 || s->queue.empty())
        return;
    const int64_t now = now_ns();
    for (size_t i = 0; i < s->queue.size();) {
        Req *q = s->queue[i];
        if (now - q->t_arr > s->cfg.queue_timeout_ns) {
            fail(s, q, OSS_E_TIMEOUT);
            s->queue.erase(s->queue.begin() + (ptrdiff_t)i);
        } else {
            ++i;
        }
    }
}

// Admit and launch queued work on free lanes, oldest request first.
void schedule(oss_server *s)
{
    expire(s);
    for (int li = 0; li < (int)s->lanes.size() && !s->queue.empty(); ++li) {
        Lane &l = s->lanes[li];
        if (l.busy)
            continue;
        Req *h = s->queue.front();
        const uint64_t key = h->r.ref_key;
        Resident *r = find_res(s, key);
        if (r && !same_desc(r->ref->desc, h->r.desc)) {
            fail(s, h, OSS_E_STATE);  // a key must always name the same image shape
            s->queue.pop_front();
            --li;
            continue;
        }
        // the tables this launch will use: the resident ones if they cover
        // every queued request on this key that joins, else new ones
        uint32_t fm = h->r.feat_mask;
        int32_t need_r = h->need_r;
        bool hit = r && (r->ref->feat_mask & fm) == fm && r->ref->max_radius >= need_r;
        if (r && !hit && r->users > 0)
            return;  // wait for the running users before replacing the tables
        std::vector<Req *> batch{h};
        int T = h->r.n_tmpl;
        for (size_t i = 1; i < s->queue.size(); ++i) {
            Req *q = s->queue[i];
            if (q->r.ref_key != key || !same_desc(q->r.desc, h->r.desc) ||
                T + q->r.n_tmpl > s->cfg.max_batch_templates)
                continue;
            if (hit && !((r->ref->feat_mask & q->r.feat_mask) == q->r.feat_mask &&
                         r->ref->max_radius >= q->need_r))
                continue;
            batch.push_back(q);
            T += q->r.n_tmpl;
        }
        if (!hit)
            for (Req *q : batch) {
                fm |= q->r.feat_mask;
                need_r = std::max(need_r, q->need_r);
            }
        if (r && !hit) {
            fm |= r->ref->feat_mask;
            need_r = std::max(need_r, r->ref->max_radius);
        }
        size_t tables = 0;
        if (!hit && oss_ref_bytes(&h->r.desc, fm, need_r, &tables) != OSS_OK) {
            fail(s, h, OSS_E_ARG);
            s->queue.pop_front();
            --li;
            continue;
        }
        // footprint: tables (unless resident), outputs, workspace growth;
        // shrink the batch from the back until it fits
        const size_t ws_now = s->lane_ws(l);
        auto need_of = [&](size_t nb) {
            int64_t tt = 0;
            size_t outs = 0;
            for (size_t i = 0; i < nb; ++i) {
                tt += batch[i]->r.n_tmpl;
                outs += batch[i]->out_bytes;
            }
            const size_t ws =
                workspace_bytes(tt, h->r.desc.H, h->r.desc.W, l.ctx->batch_bucket > 0);
            return outs + (ws > ws_now ? ws - ws_now : 0) + (hit ? 0 : tables);
        };
        // replacing non-covering tables frees them first
        if (r && !hit) {
            drop_res(s, r);
            r = nullptr;
        }
        size_t nb = batch.size();
        while (nb > 1 && !make_room(s, need_of(nb), key, hit, li))
            --nb;
        if (nb > (size_t)s->free_slots.size())
            nb = s->free_slots.size();
        if (nb == 0 || !make_room(s, need_of(nb), key, hit, li)) {
            if (!any_busy(s) && !holds_results(s)) {
                // nothing running or unreleased can free memory: never fits
                fail(s, h, OSS_E_NOMEM);
                s->queue.pop_front();
                --li;
                continue;
            }
            return;  // wait for running work to finish or results to be released
        }
        batch.resize(nb);
        r = hit ? find_res(s, key) : nullptr;  // make_room may have moved the entries
        // outputs
        bool ok = true;
        for (Req *q : batch) {
            q->out = alloc_out(s, q->out_bytes, &q->blk_bytes, l.st);
            if (!q->out) {
                ok = false;
                break;
            }
        }
        int rc = ok ? OSS_OK : OSS_E_NOMEM;
        if (rc == OSS_OK && !hit) {
            oss_ref *ref = nullptr;
            rc = oss_ref_create(l.ctx, &h->r.desc, fm, need_r, &ref);
            if (rc == OSS_OK) {
                Resident nr;
                nr.key = key;
                nr.ref = ref;
                if (hipEventCreateWithFlags(&nr.ready, hipEventDisableTiming) != hipSuccess) {
                    (void)oss_ref_release(ref);
                    rc = OSS_E_DEVICE;
                } else {
                    s->res.push_back(nr);
                    s->account((ptrdiff_t)ref->bytes);
                    r = &s->res.back();
                    s->st.builds++;
                }
            }
        }
        const int64_t t = now_ns();
        for (Req *q : batch) {
            if (rc == OSS_OK) {
                q->slot = s->free_slots.back();
                s->free_slots.pop_back();
            }
            q->batch = (int)batch.size();
            q->hit = hit ? 1 : 0;
            q->lane = li;
            q->t_launch = t;
        }
        if (rc == OSS_OK) {
            r->lru = ++s->tick;
            rc = launch(s, li, batch, r, hit);
        }
        // the batch leaves the queue whatever happened
        for (Req *q : batch)
            s->queue.erase(std::find(s->queue.begin(), s->queue.end(), q));
        if (rc != OSS_OK) {
            // enqueued work (if any) still has to finish before the slots
            // and outputs of these requests can be reused
            (void)hipStreamSynchronize(l.st);
            if (!hit) {
                // tables that may not have been built are not kept
                if (Resident *nr = find_res(s, key))
                    drop_res(s, nr);
            }
            for (Req *q : batch) {
                if (q->slot >= 0) {
                    s->free_slots.push_back(q->slot);
                    q->slot = -1;
                }
                fail(s, q, rc);
            }
            continue;
        }
        r->users++;
        l.busy = true;
        l.key = key;
        l.reqs = batch;
        s->st.launches++;
        if (hit)
            s->st.resident_hits += (int64_t)batch.size();
        for (Req *q : batch)
            q->state = RQ_RUNNING;
    }
}

}  // namespace

extern "C" {

int oss_server_create(int device, const oss_server_config *cfg, oss_server **out)
{
    if (!out || !cfg || cfg->memory_budget <= 0 || cfg->lanes < 1 || cfg->lanes > 8 ||
        cfg->max_batch_templates < 1 || cfg->queue_timeout_ns < 0)
        return OSS_E_ARG;
    *out = nullptr;
    oss_server *s = new (std::nothrow) oss_server();
    if (!s)
        return OSS_E_NOMEM;
    s->device = device;
    s->cfg = *cfg;
    int rc = OSS_OK;
    for (int i = 0; i < cfg->lanes && rc == OSS_OK; ++i) {
        Lane l;
        rc = oss_ctx_create(device, &l.ctx);
        if (rc != OSS_OK)
            break;
        if (hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess)
            rc = OSS_E_DEVICE;
        if (rc == OSS_OK) {
            // the lane's context allocates in stream order on its stream, and
            // its plan slots are sized once for the largest merged launch
            l.ctx->alloc_stream = l.st;
            rc = reserve_plan_slots(l.ctx, PLAN_RESERVE);
        }
        s->lanes.push_back(l);
    }
    if (rc == OSS_OK && hipHostMalloc(reinterpret_cast<void **>(&s->counts),
                                      COUNT_SLOTS * sizeof(int64_t), hipHostMallocDefault) !=
                            hipSuccess) {
        s->counts = nullptr;
        rc = OSS_E_NOMEM;
    }
    for (int i = COUNT_SLOTS - 1; i >= 0; --i)
        s->free_slots.push_back(i);
    if (rc != OSS_OK) {
        oss_server_destroy(s);
        return rc;
    }
    s->st.memory_budget = cfg->memory_budget;
    *out = s;
    return OSS_OK;
}

int oss_server_destroy(oss_server *s)
{
    if (!s)
        return OSS_E_ARG;
    (void)hipSetDevice(s->device);
    for (Lane &l : s->lanes)
        if (l.st)
            (void)hipStreamSynchronize(l.st);
    hipStream_t st0 = s->lanes.empty() ? nullptr : s->lanes[0].st;
    auto free_block = [&](void *p) {
        if (st0)
            (void)hipFreeAsync(p, st0);
    };
    for (auto &kv : s->reqs) {
        if (kv.second->out)
            free_block(kv.second->out);
        delete kv.second;
    }
    for (FreeBlock &b : s->cache)
        free_block(b.p);
    for (Resident &r : s->res) {
        if (r.ready)
            (void)hipEventDestroy(r.ready);
        (void)oss_ref_release(r.ref);
    }
    // each context frees its own stream-ordered buffers and waits for them,
    // before its stream goes
    for (Lane &l : s->lanes) {
        if (l.done)
            (void)hipEventDestroy(l.done);
        if (l.ctx)
            (void)oss_ctx_destroy(l.ctx);
        if (l.st) {
            (void)hipStreamSynchronize(l.st);
            (void)hipStreamDestroy(l.st);
        }
    }
    if (s->counts)
        (void)hipHostFree(s->counts);
    delete s;
    return OSS_OK;
}

int oss_server_submit(oss_server *s, const oss_request *rq, int64_t *id)
{
    if (!s || !rq || !id || !desc_ok(&rq->desc) || !rq->dev_pixels || !rq->tmpl ||
        rq->n_tmpl <= 0 || rq->n_probes < 0 || (rq->n_probes > 0 && !rq->probes) ||
        rq->list_cap < 0 || rq->feat_mask == 0 || (rq->feat_mask & ~OSS_F_ALL) ||
        rq->tol.Q <= 0)
        return OSS_E_ARG;
    for (int f = 0; f < 3; ++f)
        if ((rq->feat_mask & (1u << f)) && rq->tol.P[f] < 0)
            return OSS_E_ARG;
    for (int t = 0; t < rq->n_tmpl; ++t)
        if ((rq->tmpl[t].feat_mask & rq->feat_mask) != rq->feat_mask || rq->tmpl[t].rho < 0)
            return OSS_E_ARG;
    std::vector<int> per(rq->n_tmpl, 0);
    int32_t need_r = 0;
    for (int i = 0; i < rq->n_probes; ++i) {
        const oss_probe &p = rq->probes[i];
        if (p.template_id < 0 || p.template_id >= rq->n_tmpl || p.scale_id < 0 ||
            p.scale_id >= OSS_MAX_SCALES || p.r < 0 || ++per[p.template_id] > OSS_MAX_SCALES)
            return OSS_E_ARG;
        need_r = std::max(need_r, p.r);
    }
    if (!overflow_ok(&rq->desc, rq->feat_mask))
        return OSS_E_OVERFLOW;
    size_t tables = 0;
    int rc = oss_ref_bytes(&rq->desc, rq->feat_mask, need_r, &tables);
    if (rc != OSS_OK)
        return rc;
    // the lanes' bucket setting is the server's (fixed at create)
    const Lane &l0 = s->lanes[0];
    const size_t foot = tables + output_bytes(*rq) +
                        workspace_bytes(rq->n_tmpl, rq->desc.H, rq->desc.W,
                                        l0.ctx->batch_bucket > 0);
    if (foot > (size_t)s->cfg.memory_budget)
        return OSS_E_NOMEM;
    Req *q = new (std::nothrow) Req();
    if (!q)
        return OSS_E_NOMEM;
    q->id = s->next_id++;
    q->r = *rq;
    q->tmpl.assign(rq->tmpl, rq->tmpl + rq->n_tmpl);
    q->probes.assign(rq->probes, rq->probes + rq->n_probes);
    q->r.tmpl = nullptr;
    q->r.probes = nullptr;
    q->need_r = need_r;
    q->t_arr = rq->arrival_ns > 0 ? rq->arrival_ns : now_ns();
    q->out_bytes = output_bytes(*rq);
    s->reqs[q->id] = q;
    s->queue.push_back(q);
    s->st.submitted++;
    *id = q->id;
    return OSS_OK;
}

int oss_server_pump(oss_server *s, int64_t wait_us, int32_t *n_completed)
{
    if (!s)
        return OSS_E_ARG;
    if (hipSetDevice(s->device) != hipSuccess)
        return OSS_E_DEVICE;
    int n = retire(s);
    schedule(s);
    if (n == 0 && wait_us > 0 && any_busy(s)) {
        const int64_t end = now_ns() + wait_us * 1000;
        while (n == 0 && now_ns() < end) {
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            n = retire(s);
        }
        if (n > 0)
            schedule(s);
    }
    if (n_completed)
        *n_completed = n;
    return OSS_OK;
}

int oss_server_drain(oss_server *s)
{
    if (!s)
        return OSS_E_ARG;
    while (!s->queue.empty() || any_busy(s)) {
        int rc = oss_server_pump(s, 100000, nullptr);
        if (rc != OSS_OK)
            return rc;
        if (!s->queue.empty() && !any_busy(s))
            return OSS_E_NOMEM;  // queued work waits for results to be released
    }
    return OSS_OK;
}

int oss_server_cancel(oss_server *s, int64_t id)
{
    if (!s)
        return OSS_E_ARG;
    auto it = s->reqs.find(id);
    if (it == s->reqs.end())
        return OSS_E_ARG;
    Req *q = it->second;
    if (q->state != RQ_QUEUED)
        return OSS_E_STATE;
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), q));
    fail(s, q, OSS_E_CANCELLED);
    return OSS_OK;
}

int oss_server_result(oss_server *s, int64_t id, oss_result *out)
{
    if (!s || !out)
        return OSS_E_ARG;
    auto it = s->reqs.find(id);
    if (it == s->reqs.end())
        return OSS_E_ARG;
    const Req *q = it->second;
    std::memset(out, 0, sizeof(*out));
    out->status = (q->state == RQ_DONE || q->state == RQ_FAILED) ? q->status : OSS_E_STATE;
    out->n_tmpl = q->r.n_tmpl;
    out->H = q->r.desc.H;
    out->W = q->r.desc.W;
    out->list_cap = q->r.list_cap;
    out->batch_requests = q->batch;
    out->resident_hit = q->hit;
    out->lane = q->lane;
    if (q->state == RQ_DONE) {
        out->dev_mask = q->mask();
        out->dev_list = q->list();
        out->count = q->count;
    }
    if (q->state == RQ_DONE || q->state == RQ_FAILED) {
        out->latency_ms = (q->t_done - q->t_arr) * 1e-6;
        out->queue_ms = q->t_launch ? (q->t_launch - q->t_arr) * 1e-6 : 0.0;
    }
    return OSS_OK;
}

int oss_server_release(oss_server *s, int64_t id)
{
    if (!s)
        return OSS_E_ARG;
    auto it = s->reqs.find(id);
    if (it == s->reqs.end())
        return OSS_E_ARG;
    Req *q = it->second;
    if (q->state != RQ_DONE && q->state != RQ_FAILED)
        return OSS_E_STATE;
    if (q->out)
        s->cache.push_back({q->blk_bytes, q->out});
    s->reqs.erase(it);
    delete q;
    return OSS_OK;
}

int oss_server_stats_read(oss_server *s, oss_server_stats *out)
{
    if (!s || !out)
        return OSS_E_ARG;
    *out = s->st;
    out->bytes_in_use = (int64_t)s->in_use;
    out->bytes_peak = (int64_t)s->peak;
    out->queued = (int32_t)s->queue.size();
    int running = 0;
    for (const Lane &l : s->lanes)
        running += (int)l.reqs.size();
    out->running = running;
    return OSS_OK;
}

}  // extern "C"
