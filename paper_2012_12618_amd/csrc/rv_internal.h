// rv_internal.h -- declarations shared by the library's own source files
// (not part of the C ABI).
#ifndef RV_INTERNAL_H
#define RV_INTERNAL_H

#include <hip/hip_runtime_api.h>

#include <mutex>
#include <vector>

namespace rv_internal {
// Per-thread text returned by rv_last_error().
extern thread_local char g_error[512];
// Formats the message into g_error and returns code.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// Stage timing: while enabled, each call records kStages + 1 events around its
// kernels; rv_stage_times reads and recycles them.
constexpr int kStages = 3;
struct TimedCall {
    hipEvent_t ev[kStages + 1];
};
extern std::mutex g_timing_mutex;
extern bool g_timing;
extern std::vector<TimedCall> g_pending;  // recorded, not yet read
extern std::vector<TimedCall> g_free;     // reusable event sets
// An event set for one call, or false when timing is off.
bool take_timed_call(TimedCall &tc);
void keep_timed_call(const TimedCall &tc);
}  // namespace rv_internal

#endif
