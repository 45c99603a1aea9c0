// Online autotuner of launch choices (tile order, kernel variant, grid size)
// that leave every result unchanged: each candidate computes each output
// element with the same operations in the same order. The first launches of a
// (kernel, shape) on a device take the candidates in turn, each bracketed by
// HIP events on its stream; once every candidate has TUNE_REPS completed
// timings, the one with the smallest median is kept for the rest of the
// process and appended to the on-disk cache named by the environment
// variable GDR_TUNE_CACHE (if set), which later processes read at start-up.
// GDR_TUNE=0 turns tuning off (every site takes its default). Launches under
// HIP graph capture, and any launch while this library captures a graph in
// another thread, take the current best or the default and are not timed.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

namespace gdr {

constexpr int TUNE_REPS = 3;
constexpr int TUNE_MAXCAND = 8;

// One tunable launch: construct before the launch (choice() says which
// candidate to launch), destroy after it.
class TuneScope {
   public:
    // kernel: name of the tuning site; shape: its shape key (e.g. "24x24x24x48|12");
    // ncand candidates (<= TUNE_MAXCAND), default candidate `dflt`; work: size of
    // this launch in any unit proportional to its cost (timings are compared
    // per unit of work, so launches of one key may differ in size)
    TuneScope(const char* kernel, const std::string& shape, int ncand, int dflt, hipStream_t st,
              double work = 1.0);
    ~TuneScope();
    int choice() const { return choice_; }
    TuneScope(const TuneScope&) = delete;
    TuneScope& operator=(const TuneScope&) = delete;

   private:
    std::string key_;
    int choice_ = 0;
    hipStream_t st_ = nullptr;
    double work_ = 1.0;
    int dev_ = 0;
    hipEvent_t a_ = nullptr;   // start event while this launch is timed
};

// Load an on-disk cache (lines "v1 <kernel>|<arch>|<shape> <choice> <median us per
// unit of work>");
// malformed lines are skipped. Returns the entries taken, or -1 if unreadable.
int tune_load(const char* path);
// The decisions so far, one "kernel|arch|shape -> candidate (median us)" per line.
std::string tune_report();
// forget every decision and pending timing (tests)
void tune_reset();
// tuning enabled (GDR_TUNE is not 0)
bool tune_active();
// keys still being timed (completed timings are collected first)
int tune_open();
// keys created undecided so far (a counter that only grows)
long tune_new_open();
// Bracket a stream capture of this library: meanwhile the tuner makes no
// event call in any thread (an event query in one thread can invalidate a
// capture running in another) and launches take their decided or default form.
void tune_capture_begin();
void tune_capture_end();
struct TuneCaptureGuard {
    TuneCaptureGuard() { tune_capture_begin(); }
    ~TuneCaptureGuard() { tune_capture_end(); }
    TuneCaptureGuard(const TuneCaptureGuard&) = delete;
    TuneCaptureGuard& operator=(const TuneCaptureGuard&) = delete;
};

}  // namespace gdr
