// Per-kernel HIP-event timing (oss_ctx_profile / oss_ctx_profile_read).
#include "oss_internal.h"

namespace oss {

const char *const kKernelNames[K_COUNT] = {
    "row_base", "band_agg", "carry", "band_final",
    "star_plain", "star_batch", "compact_scan", "compact_list", "star_moments",
};

static hipEvent_t take(Profiler *p)
{
    if (!p->pool.empty()) {
        hipEvent_t e = p->pool.back();
        p->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

ProfScope::ProfScope(Profiler *p_, int id_, hipStream_t st_) : p(p_), st(st_), id(id_)
{
    if (!p || !p->on)
        return;
    // bound the number of unresolved records
    if (p->recs.size() >= 8192)
        (void)p->resolve();
    a = take(p);
    b = take(p);
    if (a && b)
        (void)hipEventRecord(a, st);
}

ProfScope::~ProfScope()
{
    if (!p || !p->on || !a || !b)
        return;
    (void)hipEventRecord(b, st);
    p->recs.push_back({id, a, b});
}

void Profiler::clear()
{
    (void)resolve();
    for (int i = 0; i < K_COUNT; ++i) {
        launches[i] = 0;
        total_ms[i] = 0.0;
        max_ms[i] = 0.0;
    }
}

hipError_t Profiler::resolve()
{
    hipError_t err = hipSuccess;
    for (const Rec &r : recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e == hipSuccess) {
            launches[r.id] += 1;
            total_ms[r.id] += ms;
            if (ms > max_ms[r.id])
                max_ms[r.id] = ms;
        } else {
            err = e;
        }
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    recs.clear();
    return err;
}

Profiler::~Profiler()
{
    (void)resolve();
    for (hipEvent_t e : pool)
        (void)hipEventDestroy(e);
}

}  // namespace oss
