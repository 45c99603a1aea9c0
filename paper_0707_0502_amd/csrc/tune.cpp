// Online autotuner (see tune.h).
#include "tune.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

namespace gdr {
namespace {

struct Entry {
    int ncand = 0;
    int best = -1;                                 // decided candidate, -1 while tuning
    double best_us = 0;
    std::vector<std::vector<float>> ms;            // completed timings per candidate
    std::vector<int> issued;                       // timings issued per candidate
    int next = 0;                                  // next candidate to time
};

struct Pending {
    std::string key;
    int cand;
    double work;
    int dev;
    hipEvent_t a, b;
};

struct State {
    std::mutex mu;
    bool loaded = false;
    bool enabled = true;
    std::string cache;                             // GDR_TUNE_CACHE
    std::map<std::string, Entry> table;
    std::map<std::string, std::pair<int, double>> stored;   // from the cache file
    std::vector<Pending> pend;
    std::map<int, std::vector<hipEvent_t>> pool;   // idle events per device
    std::map<int, std::string> arch;               // architecture name per device
    long new_open = 0;                             // keys created undecided
    int capturing = 0;                             // stream captures in progress
};

State& S() {
    static State s;
    return s;
}

std::string arch_name(State& s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    auto it = s.arch.find(dev);
    if (it != s.arch.end()) return it->second;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    if (c != std::string::npos) a = a.substr(0, c);
    s.arch[dev] = a;
    return a;
}

int load_locked(State& s, const char* path) {
    FILE* f = std::fopen(path, "r");
    if (!f) return -1;
    char line[1024];
    int taken = 0;
    while (std::fgets(line, sizeof line, f)) {
        char ver[8], key[900];
        int choice = -1;
        double us = 0;
        if (std::sscanf(line, "%7s %899s %d %lf", ver, key, &choice, &us) != 4) continue;
        if (std::strcmp(ver, "v1") != 0 || choice < 0 || choice >= TUNE_MAXCAND || !(us >= 0))
            continue;
        s.stored[key] = {choice, us};
        ++taken;
    }
    std::fclose(f);
    return taken;
}

void ensure_loaded(State& s) {
    if (s.loaded) return;
    s.loaded = true;
    const char* t = std::getenv("GDR_TUNE");
    if (t && std::strcmp(t, "0") == 0) s.enabled = false;
    const char* c = std::getenv("GDR_TUNE_CACHE");
    if (c && *c) {
        s.cache = c;
        (void)load_locked(s, c);
    }
}

// an idle event of device dev (the current device)
hipEvent_t get_event(State& s, int dev) {
    auto& v = s.pool[dev];
    if (!v.empty()) {
        hipEvent_t e = v.back();
        v.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;   // error left for the caller's check
    return e;
}

void decide(State& s, const std::string& key, Entry& e) {
    double best = 1e300;
    int bi = 0;
    for (int c = 0; c < e.ncand; ++c) {
        std::vector<float> v = e.ms[c];
        std::sort(v.begin(), v.end());
        const double med = v[v.size() / 2];
        if (med < best) {
            best = med;
            bi = c;
        }
    }
    e.best = bi;
    e.best_us = best * 1e3;
    if (!s.cache.empty()) {
        FILE* f = std::fopen(s.cache.c_str(), "a");
        if (f) {
            std::fprintf(f, "v1 %s %d %.3f\n", key.c_str(), bi, e.best_us);
            std::fclose(f);
        }
    }
}

// completed timings into their entries (events not yet done stay pending).
// Skipped while an error is pending on this thread, so that clearing the
// not-ready status of a query never hides an earlier launch error.
void harvest(State& s) {
    if (s.pend.empty() || s.capturing > 0 || hipPeekAtLastError() != hipSuccess) return;
    std::vector<Pending> keep;
    for (auto& p : s.pend) {
        const hipError_t q = hipEventQuery(p.b);
        if (q != hipSuccess) {
            (void)hipGetLastError();
            keep.push_back(p);
            continue;
        }
        float ms = 0;
        const bool ok = hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess;
        if (!ok) (void)hipGetLastError();
        auto it = s.table.find(p.key);
        if (!ok && it != s.table.end() && it->second.best < 0) --it->second.issued[p.cand];
        if (ok && it != s.table.end() && it->second.best < 0) {
            Entry& e = it->second;
            e.ms[p.cand].push_back((float)(ms / p.work));
            bool done = true;
            for (int c = 0; c < e.ncand; ++c) done = done && (int)e.ms[c].size() >= TUNE_REPS;
            if (done) decide(s, p.key, e);
        }
        s.pool[p.dev].push_back(p.a);
        s.pool[p.dev].push_back(p.b);
    }
    s.pend.swap(keep);
}

}  // namespace

TuneScope::TuneScope(const char* kernel, const std::string& shape, int ncand, int dflt,
                     hipStream_t st, double work)
    : st_(st), work_(work > 0 ? work : 1.0) {
    choice_ = (dflt >= 0 && dflt < ncand) ? dflt : 0;
    if (ncand <= 1 || ncand > TUNE_MAXCAND) return;
    // Under stream capture only capture-safe calls are made: no event query or
    // record, no device-property query (they would invalidate the capture).
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess) return;   // error left for the caller

    const bool capturing = cap != hipStreamCaptureStatusNone;
    State& s = S();
    std::lock_guard<std::mutex> g(s.mu);
    ensure_loaded(s);
    if (!s.enabled) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    if (capturing && s.arch.find(dev) == s.arch.end()) return;
    key_ = std::string(kernel) + "|" + arch_name(s) + "|" + shape;
    if (!capturing) harvest(s);
    auto it = s.table.find(key_);
    if (it == s.table.end()) {
        Entry e;
        e.ncand = ncand;
        e.ms.assign(ncand, {});
        e.issued.assign(ncand, 0);
        auto st_it = s.stored.find(key_);
        if (st_it != s.stored.end() && st_it->second.first < ncand) {
            e.best = st_it->second.first;
            e.best_us = st_it->second.second;
        } else {
            ++s.new_open;
        }
        it = s.table.emplace(key_, e).first;
    }
    Entry& e = it->second;
    if (e.ncand != ncand) return;   // same key used with another candidate count: default
    if (e.best >= 0) {
        choice_ = e.best;
        return;
    }
    // graph capture here or in another thread: default, not timed
    if (capturing || s.capturing > 0) return;
    // candidates in turn, TUNE_REPS timings each; launches issued while the
    // last timings are still in flight take the default
    int c = -1;
    for (int t = 0; t < ncand && c < 0; ++t) {
        const int q = (e.next + t) % ncand;
        if (e.issued[q] < TUNE_REPS) c = q;
    }
    if (c < 0) return;
    a_ = get_event(s, dev);
    if (!a_) return;                                       // error left for the caller's check
    if (hipEventRecord(a_, st) != hipSuccess) {            // error left for the caller's check
        s.pool[dev].push_back(a_);
        a_ = nullptr;
        return;
    }
    choice_ = c;
    dev_ = dev;
    e.next = (c + 1) % ncand;
    ++e.issued[c];
}

TuneScope::~TuneScope() {
    if (!a_) return;
    State& s = S();
    std::lock_guard<std::mutex> g(s.mu);
    auto untime = [&] {   // this timing will not complete: its slot is issued again
        auto it = s.table.find(key_);
        if (it != s.table.end() && it->second.best < 0) --it->second.issued[choice_];
    };
    if (s.capturing > 0) {   // a capture began meanwhile: drop this timing
        s.pool[dev_].push_back(a_);
        untime();
        return;
    }
    hipEvent_t b = get_event(s, dev_);
    if (!b || hipEventRecord(b, st_) != hipSuccess) {   // error left for the caller's check
        s.pool[dev_].push_back(a_);
        if (b) s.pool[dev_].push_back(b);
        untime();
        return;
    }
    s.pend.push_back({key_, choice_, work_, dev_, a_, b});
}

int tune_load(const char* path) {
    State& s = S();
    std::lock_guard<std::mutex> g(s.mu);
    ensure_loaded(s);
    if (!path) return -1;
    return load_locked(s, path);
}

std::string tune_report() {
    State& s = S();
    std::lock_guard<std::mutex> g(s.mu);
    ensure_loaded(s);
    harvest(s);
    std::string out;
    char buf[64];
    for (auto& kv : s.table) {
        if (kv.second.best < 0) continue;
        std::snprintf(buf, sizeof buf, " -> %d (%.3g us per unit)\n", kv.second.best,
                      kv.second.best_us);
        out += kv.first + buf;
    }
    return out;
}

void tune_reset() {
    State& s = S();
    std::lock_guard<std::mutex> g(s.mu);
    for (auto& p : s.pend) {
        (void)hipEventSynchronize(p.b);
        s.pool[p.dev].push_back(p.a);
        s.pool[p.dev].push_back(p.b);
    }
    s.pend.clear();
    s.table.clear();
    s.stored.clear();
    s.loaded = false;
}

bool tune_active() {
    State& s = S();
    std::lock_guard<std::mutex> g(s.mu);
    ensure_loaded(s);
    return s.enabled;
}

int tune_open() {
    State& s = S();
    std::lock_guard<std::mutex> g(s.mu);
    harvest(s);
    int k = 0;
    for (auto& kv : s.table) k += kv.second.best < 0;
    return k;
}

long tune_new_open() {
    State& s = S();
    std::lock_guard<std::mutex> g(s.mu);
    return s.new_open;
}

void tune_capture_begin() {
    State& s = S();
    std::lock_guard<std::mutex> g(s.mu);
    ++s.capturing;
}

void tune_capture_end() {
    State& s = S();
    std::lock_guard<std::mutex> g(s.mu);
    --s.capturing;
}

}  // namespace gdr
