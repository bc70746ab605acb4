// log.h -- diagnostic lines on stderr, chosen by the SELLCS_LOG environment variable (read
// once per process): unset or 0 prints nothing; 1 prints performance warnings (a call that
// runs a slower kernel than its operands' shape would need); 2 also prints what builds and
// tuning decide. Lines start with "[sellcs] PERFWARNING " or "[sellcs] INFO ", after the
// warning and information lines of the benchmark runs in Sec. 4.1.
#pragma once

namespace sellcs {

// what a performance warning is about: each is printed once per process
enum LogWarn {
    kWarnProductWidth = 0,   // a block width with no fixed-width kernel
    kWarnProductLayout = 1,  // column-major, strided or unaligned block vectors
    kWarnBatchGeneral = 2,   // the same, in a batched product
    kWarnAtomicTranspose = 3,
    kWarnCount = 8
};

int log_level();
void log_info(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void log_warn_once(LogWarn what, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

}  // namespace sellcs
