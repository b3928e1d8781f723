// Kernel timing hooks: when enabled, every instrumented launch is bracketed
// by a pair of HIP events recorded on the launch's own stream (or, for a
// launch made with hipExtLaunchKernelGGL, recorded by its dispatch), and the
// elapsed times are summed per kernel class when profiling ends.  Disabled by
// default; enabling it adds two event records per launch and no
// synchronisation until husky_profile_end.

#include <mutex>
#include <vector>

#include "../../include/husky.h"
#include "internal.h"

namespace husky {
namespace {

struct Pair {
    hipEvent_t a, b;
    int cls;
};

std::mutex g_mu;
bool g_on = false;
uint32_t g_mask = ~0u;  // kernel classes to bracket
std::vector<Pair> g_used;
std::vector<Pair> g_free;

}  // namespace

bool prof_on() { return g_on; }

ProfScope::ProfScope(int cls, hipStream_t s) : cls_(cls), s_(s), idx_(-1) {
    if (!g_on || cls < 0 || cls >= 32 || !((g_mask >> cls) & 1u)) return;
    std::lock_guard<std::mutex> lk(g_mu);
    Pair p;
    if (!g_free.empty()) {
        p = g_free.back();
        g_free.pop_back();
    } else {
        if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) return;
    }
    p.cls = cls;
    if (hipEventRecord(p.a, s) != hipSuccess) {
        g_free.push_back(p);
        return;
    }
    g_used.push_back(p);
    idx_ = (int)g_used.size() - 1;
}

ProfScope::ProfScope(int cls, hipStream_t s, hipEvent_t* start, hipEvent_t* stop)
    : cls_(cls), s_(s), idx_(-1), deferred_(true) {
    *start = *stop = nullptr;
    if (!g_on || cls < 0 || cls >= 32 || !((g_mask >> cls) & 1u)) return;
    std::lock_guard<std::mutex> lk(g_mu);
    Pair p;
    if (!g_free.empty()) {
        p = g_free.back();
        g_free.pop_back();
    } else {
        if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) return;
    }
    p.cls = cls;
    g_used.push_back(p);
    idx_ = (int)g_used.size() - 1;
    *start = p.a;
    *stop = p.b;
}

ProfScope::~ProfScope() {
    if (idx_ < 0 || deferred_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    (void)hipEventRecord(g_used[idx_].b, s_);
}

}  // namespace husky

using namespace husky;

extern "C" {

void husky_profile_select(uint32_t class_mask) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_mask = class_mask;
}

void husky_profile_begin(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& p : g_used) g_free.push_back(p);
    g_used.clear();
    g_on = true;
}

int husky_profile_end(double* ms, uint32_t* launches, int n_classes) {
    std::vector<Pair> used;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_on = false;
        used.swap(g_used);
    }
    for (int c = 0; c < n_classes; ++c) {
        ms[c] = 0.0;
        launches[c] = 0;
    }
    int rc = 0;
    for (auto& p : used) {
        if (hipEventSynchronize(p.b) != hipSuccess) {
            rc = HUSKY_ERR_HIP;
            continue;
        }
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.a, p.b) != hipSuccess) {
            rc = HUSKY_ERR_HIP;
            continue;
        }
        if (p.cls >= 0 && p.cls < n_classes) {
            ms[p.cls] += t;
            launches[p.cls] += 1;
        }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& p : used) g_free.push_back(p);
    return rc;
}

}  // extern "C"
