// The tuner's search machinery, independent of the kernel being tuned: a
// measurer interface (compile a set of configurations, then verify and time
// one), the exhaustive sweep over a candidate list, and the final re-timing
// and tie-broken choice of the winner (Section 3 of the paper: compile and
// benchmark every point of a restricted space; Section 4: tuning impact).
// The convolution tuner and the hotspot tuner both run on it.
#pragma once

#include <algorithm>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

namespace conv2d {

enum MeasureStatus { kOk = 0, kCompile = CONV2D_ECOMPILE, kLaunch = CONV2D_ELAUNCH, kVerify = CONV2D_EVERIFY };
const char* status_name(int s);
int status_from(const std::string& n);
// numpy's median (mean of the two middle values for an even count)
double median_of(std::vector<double> v);
// nearest-rank quantile, p in [0, 1]
double quantile_nearest(std::vector<double> v, double p);

template <class Cfg>
struct RecordT {
    Cfg c{};
    int status = kOk;
    double ms = 0, ms_min = 0, ms_p90 = 0;   // median, minimum, p90 of the timed launches
    int reps = 0;
};

template <class Cfg>
class MeasurerT {
public:
    virtual ~MeasurerT() = default;
    virtual std::string arch() const = 0;
    // Compile (or otherwise prepare) every config; status[i] gets kOk or a failure.
    virtual int prepare(const std::vector<Cfg>& cfgs, std::vector<int>* status, double* seconds) = 0;
    // Verify and time one prepared config (reps timed launches); best_so_far
    // (0: none) lets a far slower point stop early.
    virtual int measure(const Cfg& c, int warmup, int reps, double best_so_far, RecordT<Cfg>* r) = 0;
    // Sustained timing for later measure() calls: the reps launches run back
    // to back, as an application runs them, cycling through copies of the
    // data larger together than the last-level cache so that every launch
    // starts cold, and the mean is taken. Off: each launch is timed alone
    // after a cache flush.
    virtual void set_sustained(bool on) { (void)on; }
};

// Prepares and measures every configuration of `todo`, storing each record in
// `done` under key(c) and passing it to sink(record). *best follows the
// fastest verified time (0 = none yet); *compile_s accumulates compile time.
template <class Cfg, class Key, class Sink>
int measure_all(const std::vector<Cfg>& todo, MeasurerT<Cfg>* m, int warmup, int reps, bool verbose, Key key,
                Sink sink, std::map<std::string, RecordT<Cfg>>* done, double* best, double* compile_s)
{
    std::vector<int> status;
    double sec = 0;
    int rc = m->prepare(todo, &status, &sec);
    if (rc) return rc;
    if (compile_s) *compile_s += sec;
    for (size_t i = 0; i < todo.size(); ++i) {
        RecordT<Cfg> r;
        r.c = todo[i];
        if (status[i] != kOk) {
            r.status = status[i];
        } else {
            rc = m->measure(todo[i], warmup, reps, *best, &r);
            if (rc) return rc;
            if (r.status == kOk && (*best == 0 || r.ms < *best)) *best = r.ms;
        }
        (*done)[key(r.c)] = r;
        sink(r);
        if (verbose && ((i + 1) % 100 == 0 || i + 1 == todo.size()))
            std::fprintf(stderr, "[tune] measured %zu/%zu, best %.4f ms\n", i + 1, todo.size(), *best);
    }
    return CONV2D_OK;
}

// Sorts `eligible` (verified records of the sweep) by time, ties by less();
// re-times the n_top fastest with retime_reps sustained launches (0: keeps
// the sweep's times) into *top, sorted by the new time; the winner is the
// smallest configuration under less() among those within tie_rel of the
// fastest of *top. Only re-timed points compete: the sweep times a launch
// alone after a cache flush, which favours configurations that do well in
// bursts, while applications run launches back to back.
template <class Cfg, class Less>
int retime_and_pick(std::vector<RecordT<Cfg>>* eligible, MeasurerT<Cfg>* m, int warmup, int retime_reps,
                    int n_top, double tie_rel, Less less, std::vector<RecordT<Cfg>>* top, RecordT<Cfg>* win)
{
    if (eligible->empty()) return fail(CONV2D_EVERIFY, "no configuration compiled, ran and verified");
    auto by_time = [&](const RecordT<Cfg>& a, const RecordT<Cfg>& b) {
        return a.ms != b.ms ? a.ms < b.ms : less(a.c, b.c);
    };
    std::sort(eligible->begin(), eligible->end(), by_time);
    n_top = std::max(1, std::min<int>(n_top, (int)eligible->size()));
    top->assign(eligible->begin(), eligible->begin() + n_top);
    if (retime_reps > 0) {
        std::vector<Cfg> cfgs;
        for (const auto& r : *top) cfgs.push_back(r.c);
        std::vector<int> st;
        double sec = 0;
        int rc = m->prepare(cfgs, &st, &sec);
        if (rc) return rc;
        m->set_sustained(true);
        std::vector<RecordT<Cfg>> timed;
        for (int k = 0; k < n_top && rc == CONV2D_OK; ++k) {
            if (st[k] != kOk) continue;
            RecordT<Cfg> r;
            rc = m->measure(cfgs[k], warmup, retime_reps, 0, &r);
            if (rc == CONV2D_OK && r.status == kOk) timed.push_back(r);
        }
        m->set_sustained(false);
        if (rc) return rc;
        if (timed.empty()) return fail(CONV2D_EVERIFY, "re-timing: no configuration ran and verified");
        *top = timed;
    }
    std::sort(top->begin(), top->end(), by_time);
    const double fastest = (*top)[0].ms;
    *win = (*top)[0];
    for (const auto& r : *top)
        if (r.ms <= fastest * (1.0 + tie_rel) && less(r.c, win->c)) *win = r;
    return CONV2D_OK;
}

// Times one configuration the way retime_and_pick times its candidates
// (retime_reps sustained launches), so that a baseline such as the default
// configuration can be compared with the winner in the same timing mode.
// *r keeps the status of a failure; returns a non-zero status only for an
// error of the measurer itself.
template <class Cfg>
int retime_one(const Cfg& c, MeasurerT<Cfg>* m, int warmup, int retime_reps, RecordT<Cfg>* r)
{
    std::vector<int> st;
    double sec = 0;
    int rc = m->prepare({c}, &st, &sec);
    if (rc) return rc;
    r->c = c;
    if (st[0] != kOk) {
        r->status = st[0];
        return CONV2D_OK;
    }
    m->set_sustained(true);
    rc = m->measure(c, warmup, retime_reps, 0, r);
    m->set_sustained(false);
    return rc;
}

}  // namespace conv2d
