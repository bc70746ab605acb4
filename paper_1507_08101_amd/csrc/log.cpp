// log.cpp -- the SELLCS_LOG diagnostic lines (levels in log.h).
#include "log.h"

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <mutex>

namespace sellcs {

namespace {
std::mutex g_out;
std::atomic<bool> g_warned[kWarnCount];

void emit(const char *tag, const char *fmt, va_list ap) {
    std::lock_guard<std::mutex> lk(g_out);
    std::fprintf(stderr, "[sellcs] %s ", tag);
    std::vfprintf(stderr, fmt, ap);
    std::fputc('\n', stderr);
    std::fflush(stderr);
}
}  // namespace

int log_level() {
    static const int level = [] {
        const char *e = std::getenv("SELLCS_LOG");
        const int v = e ? std::atoi(e) : 0;
        return v < 0 ? 0 : v;
    }();
    return level;
}

void log_info(const char *fmt, ...) {
    if (log_level() < 2) return;
    va_list ap;
    va_start(ap, fmt);
    emit("INFO", fmt, ap);
    va_end(ap);
}

void log_warn_once(LogWarn what, const char *fmt, ...) {
    if (log_level() < 1 || what < 0 || what >= kWarnCount) return;
    if (g_warned[what].exchange(true)) return;
    va_list ap;
    va_start(ap, fmt);
    emit("PERFWARNING", fmt, ap);
    va_end(ap);
}

}  // namespace sellcs
