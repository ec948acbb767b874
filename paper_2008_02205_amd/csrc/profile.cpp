// Event timing of kernel classes for roofline reports (mlpg_profile_*).
#include <vector>

#include <atomic>

#include "internal.hpp"

namespace mlpg {

namespace {

struct Rec {
    int cls;
    double bytes;
    hipEvent_t a, b;
};

// At most this many launches of a class are bracketed per profiling session
// (the first ones): enough for a per-launch average, and a bounded number of
// events however long the profiled work is.
constexpr int64_t kMaxPerClass = 4096;

struct State {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<Rec> recs;
    size_t used = 0;
    int64_t per_class[MLPG_PROF_CLASSES] = {};
};

State g_prof;

hipEvent_t take()
{
    if (g_prof.used < g_prof.pool.size()) return g_prof.pool[g_prof.used++];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_prof.pool.push_back(e);
    g_prof.used++;
    return e;
}

}  // namespace

bool prof_on() { return g_prof.on; }

int prof_start(int cls, double bytes, hipStream_t s)
{
    if (!g_prof.on || cls < 0 || cls >= MLPG_PROF_CLASSES || g_prof.per_class[cls] >= kMaxPerClass) return -1;
    g_prof.per_class[cls]++;
    Rec r{cls, bytes, take(), take()};
    if (!r.a || !r.b || hipEventRecord(r.a, s) != hipSuccess) return -1;
    g_prof.recs.push_back(r);
    return (int)g_prof.recs.size() - 1;
}

void prof_stop(int id, hipStream_t s)
{
    if (id < 0) return;
    (void)hipEventRecord(g_prof.recs[id].b, s);
}

}  // namespace mlpg

using namespace mlpg;

extern "C" int mlpg_profile_begin(void)
{
    g_prof.on = true;
    g_prof.recs.clear();
    g_prof.used = 0;
    for (int c = 0; c < MLPG_PROF_CLASSES; ++c) g_prof.per_class[c] = 0;
    return MLPG_OK;
}

extern "C" int mlpg_profile_end(double *ms, int64_t *launches, double *bytes)
{
    MLPG_CHECK(ms && launches && bytes, MLPG_ERR_ARG, "mlpg_profile_end: null output");
    for (int c = 0; c < MLPG_PROF_CLASSES; ++c) {
        ms[c] = 0.0;
        launches[c] = 0;
        bytes[c] = 0.0;
    }
    g_prof.on = false;
    MLPG_HIP(hipDeviceSynchronize());
    for (const Rec &r : g_prof.recs) {
        float t = 0.0f;
        MLPG_HIP(hipEventElapsedTime(&t, r.a, r.b));
        if (r.cls < 0 || r.cls >= MLPG_PROF_CLASSES) continue;
        ms[r.cls] += t;
        launches[r.cls] += 1;
        bytes[r.cls] += r.bytes;
    }
    g_prof.recs.clear();
    g_prof.used = 0;
    return MLPG_OK;
}

namespace mlpg {
namespace {
std::atomic<mlpg_progress_fn> g_progress{nullptr};
std::atomic<void *> g_progress_user{nullptr};
}  // namespace

void report_progress(int level, int64_t iters, double resid)
{
    mlpg_progress_fn fn = g_progress.load();
    if (fn) fn(g_progress_user.load(), level, iters, resid);
}
}  // namespace mlpg

extern "C" int mlpg_set_progress(mlpg_progress_fn fn, void *user)
{
    mlpg::g_progress_user.store(user);
    mlpg::g_progress.store(fn);
    return MLPG_OK;
}
