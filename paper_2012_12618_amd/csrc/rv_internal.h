// rv_internal.h -- declarations shared by the library's own source files
// (not part of the C ABI).
#ifndef RV_INTERNAL_H
#define RV_INTERNAL_H

namespace rv_internal {
// Per-thread text returned by rv_last_error().
extern thread_local char g_error[512];
// Formats the message into g_error and returns code.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
}  // namespace rv_internal

#endif
