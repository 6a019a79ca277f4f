// Per-kernel timing with HIP events recorded on the stream each kernel is
// launched on: while a profile is open, every launch of a selected kind is
// bracketed by a pair of events from a pool created when the profile opens,
// so no allocation happens between the launches being timed.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "fd_internal.h"

namespace fd {
namespace {

struct ProfState {
    std::mutex m;
    std::atomic<bool> on{false};
    unsigned mask = 0;
    int device = -1;
    std::vector<hipEvent_t> ev;      // 2 per slot: start, end
    std::vector<int> kind;           // per used slot
    int used = 0;
    int64_t dropped = 0;             // launches of a selected kind past the pool
};

ProfState& prof() {
    static ProfState s;
    return s;
}

void destroy_events(ProfState& s) {
    for (hipEvent_t e : s.ev) (void)hipEventDestroy(e);
    s.ev.clear();
    s.kind.clear();
    s.used = 0;
}

}  // namespace

int prof_begin(int kind, hipStream_t st) {
    ProfState& s = prof();
    if (!s.on.load(std::memory_order_relaxed)) return -1;   // the common case: no profile open
    std::lock_guard<std::mutex> g(s.m);
    if (!s.on || !(s.mask & (1u << kind))) return -1;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != s.device) return -1;
    if (s.used >= (int)s.kind.size()) {
        ++s.dropped;
        return -1;
    }
    const int slot = s.used++;
    s.kind[slot] = kind;
    if (hipEventRecord(s.ev[2 * slot], st) != hipSuccess) s.kind[slot] = -1;
    return slot;
}

void prof_end(int slot, hipStream_t st) {
    if (slot < 0) return;
    ProfState& s = prof();
    std::lock_guard<std::mutex> g(s.m);
    if (hipEventRecord(s.ev[2 * slot + 1], st) != hipSuccess) s.kind[slot] = -1;
}

}  // namespace fd

using namespace fd;

extern "C" {

fd_status fd_profile_begin(uint32_t kind_mask, int32_t max_launches) {
    if (max_launches <= 0 || max_launches > (1 << 20) || kind_mask == 0 || (kind_mask >> FD_PROF_KINDS))
        return FD_EINVAL;
    ProfState& s = prof();
    std::lock_guard<std::mutex> g(s.m);
    if (s.on) return FD_EINVAL;                  // one profile at a time
    destroy_events(s);
    if (hipGetDevice(&s.device) != hipSuccess) return FD_EHIP;
    s.ev.resize(2 * (size_t)max_launches, nullptr);
    for (auto& e : s.ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            destroy_events(s);
            return FD_EHIP;
        }
    }
    s.kind.assign(max_launches, -1);
    s.used = 0;
    s.dropped = 0;
    s.mask = kind_mask;
    s.on = true;
    return FD_OK;
}

fd_status fd_profile_end(double* total_ms, int64_t* launches, double* min_ms, double* max_ms, int64_t* dropped) {
    ProfState& s = prof();
    std::lock_guard<std::mutex> g(s.m);
    if (!s.on) return FD_EINVAL;
    s.on = false;
    fd_status rc = FD_OK;
    for (int k = 0; k < FD_PROF_KINDS; ++k) {
        if (total_ms) total_ms[k] = 0.0;
        if (launches) launches[k] = 0;
        if (min_ms) min_ms[k] = 0.0;
        if (max_ms) max_ms[k] = 0.0;
    }
    for (int i = 0; i < s.used; ++i) {
        const int k = s.kind[i];
        if (k < 0) continue;
        if (hipEventSynchronize(s.ev[2 * i + 1]) != hipSuccess) {
            rc = FD_EHIP;
            break;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, s.ev[2 * i], s.ev[2 * i + 1]) != hipSuccess) {
            rc = FD_EHIP;
            break;
        }
        if (launches && total_ms) {
            if (min_ms && (launches[k] == 0 || ms < min_ms[k])) min_ms[k] = ms;
            if (max_ms && ms > max_ms[k]) max_ms[k] = ms;
            total_ms[k] += ms;
            launches[k] += 1;
        }
    }
    if (dropped) *dropped = s.dropped;
    destroy_events(s);
    return rc;
}

}  // extern "C"
