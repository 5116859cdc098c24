// timing.hip -- optional HIP-event timing of every kernel launch the library enqueues (the
// measurement hook of include/pplace.h).  Off by default; when on, each launch site records a
// start and a stop event on the caller's stream, tagged with its stage name.
#include <mutex>
#include <string.h>
#include <vector>

#include "../../include/pplace.h"
#include "common.h"

namespace pp {
namespace {

struct Rec {
    const char *name;
    hipEvent_t start, stop;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;

void clear_locked() {
    for (Rec &r : g_recs) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    g_recs.clear();
}

}  // namespace

TimedLaunch::TimedLaunch(const char *name, hipStream_t s) : name_(name), s_(s) {
    if (!name) return;   // an untimed launch site
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    if (hipEventCreate((hipEvent_t *)&start_) != hipSuccess) return;
    if (hipEventCreate((hipEvent_t *)&stop_) != hipSuccess) {
        (void)hipEventDestroy((hipEvent_t)start_);
        start_ = nullptr;
        return;
    }
    (void)hipEventRecord((hipEvent_t)start_, s_);
    active_ = true;
}

TimedLaunch::~TimedLaunch() {
    if (!active_) return;
    (void)hipEventRecord((hipEvent_t)stop_, s_);
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.push_back(Rec{name_, (hipEvent_t)start_, (hipEvent_t)stop_});
}

}  // namespace pp

using namespace pp;

extern "C" {

int pp_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    clear_locked();
    g_on = on != 0;
    return PP_OK;
}

int pp_timing_query(const char *name, double *total_ms, int *count) {
    if (!name || !total_ms || !count) return PP_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    double tot = 0.0;
    int c = 0;
    for (const Rec &r : g_recs) {
        if (strcmp(r.name, name) != 0) continue;
        if (hipEventSynchronize(r.stop) != hipSuccess) return PP_ERR_DEVICE;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return PP_ERR_DEVICE;
        tot += ms;
        ++c;
    }
    *total_ms = tot;
    *count = c;
    return PP_OK;
}

}  // extern "C"
