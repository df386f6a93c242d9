// The auto-tuner: enumerate the restricted space, compile every point in
// parallel, verify each bitwise against the reference kernel, time it with
// HIP events, pick the winner, report the paper's tuning impact (best over
// median throughput, Section 4 and Table 3) and the tuned/default speedup,
// and cache the winner per (arch, shape, kernel source).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <memory>
#include <set>
#include <thread>

#include "internal.h"
#include "search.h"

namespace conv2d {

// ---------------------------------------------------------------- winners cache

std::string winners_default_path() { return library_dir() + "/tuned/winners.jsonl"; }

static std::string shape_json(const conv2d_shape& s)
{
    char b[96];
    std::snprintf(b, sizeof b, "[%d,%d,%d,%d]", s.out_h, s.out_w, s.filt_h, s.filt_w);
    return b;
}

static std::string config_json(const conv2d_config& c) { return "[" + config_str(c) + "]"; }

static bool json_shape_is(const JsonObj& o, const conv2d_shape& s)
{
    auto it = o.arr.find("shape");
    if (it == o.arr.end() || it->second.size() != 4) return false;
    const auto& a = it->second;
    return (int)a[0] == s.out_h && (int)a[1] == s.out_w && (int)a[2] == s.filt_h && (int)a[3] == s.filt_w;
}

static bool json_config(const JsonObj& o, conv2d_config* c)
{
    auto it = o.arr.find("config");
    if (it == o.arr.end() || it->second.size() != 7) return false;
    const auto& a = it->second;
    *c = conv2d_config{(int)a[0], (int)a[1], (int)a[2], (int)a[3], (int)a[4], (int)a[5], (int)a[6]};
    return true;
}

// An entry tuned for the current kernel source wins; an entry for an older
// source revision of the same (arch, shape) is used only when no current one
// exists (every configuration is correct; it may no longer be the fastest).
int cache_lookup(const std::string& path, const std::string& arch, const conv2d_shape& s,
                 conv2d_config* c, double* ms, bool* stale)
{
    std::ifstream f(path);
    if (!f) return fail(CONV2D_ENOTUNED, "no winners cache at " + path);
    const std::string src = hex64(direct_source_hash());
    bool have_cur = false, have_old = false;
    conv2d_config cur{}, old{};
    double cur_ms = 0, old_ms = 0;
    std::string line;
    while (std::getline(f, line)) {
        JsonObj o;
        if (!json_parse_line(line, &o)) continue;
        if (o.str["arch"] != arch || !json_shape_is(o, s)) continue;
        conv2d_config cc;
        if (!json_config(o, &cc)) continue;
        if (o.str["src"] == src) { cur = cc; cur_ms = o.num["ms"]; have_cur = true; }
        else { old = cc; old_ms = o.num["ms"]; have_old = true; }
    }
    if (!have_cur && !have_old) return fail(CONV2D_ENOTUNED, "shape not in winners cache");
    if (c) *c = have_cur ? cur : old;
    if (ms) *ms = have_cur ? cur_ms : old_ms;
    if (stale) *stale = !have_cur;
    return CONV2D_OK;
}

int cache_lookup_filter(const std::string& path, const std::string& arch, int fh, int fw,
                        const conv2d_shape& prefer, conv2d_config* c)
{
    if (cache_lookup(path, arch, prefer, c, nullptr) == CONV2D_OK) return CONV2D_OK;
    std::ifstream f(path);
    if (!f) return fail(CONV2D_ENOTUNED, "no winners cache at " + path);
    const std::string src = hex64(direct_source_hash());
    bool have_cur = false, have_old = false;
    conv2d_config cur{}, old{};
    std::string line;
    while (std::getline(f, line)) {
        JsonObj o;
        if (!json_parse_line(line, &o) || o.str["arch"] != arch) continue;
        auto it = o.arr.find("shape");
        if (it == o.arr.end() || it->second.size() != 4 || (int)it->second[2] != fh || (int)it->second[3] != fw)
            continue;
        conv2d_config cc;
        if (!json_config(o, &cc)) continue;
        if (o.str["src"] == src) { cur = cc; have_cur = true; }
        else { old = cc; have_old = true; }
    }
    if (!have_cur && !have_old) return fail(CONV2D_ENOTUNED, "filter size not in winners cache");
    *c = have_cur ? cur : old;
    return CONV2D_OK;
}

int cache_store(const std::string& path, const std::string& arch, const conv2d_shape& s,
                const conv2d_config& c, double ms)
{
    size_t k = path.find_last_of('/');
    if (k != std::string::npos) make_dirs(path.substr(0, k));
    char b[512];
    std::snprintf(b, sizeof b,
                  "{\"arch\":\"%s\",\"src\":\"%s\",\"shape\":%s,\"config\":%s,\"ms\":%.6f}",
                  json_escape(arch).c_str(), hex64(direct_source_hash()).c_str(), shape_json(s).c_str(),
                  config_json(c).c_str(), ms);
    if (!append_line(path, b)) return fail(CONV2D_EINVAL, "cannot write winners cache " + path);
    return CONV2D_OK;
}

namespace {

// ---------------------------------------------------------------- records

using Record = RecordT<conv2d_config>;

}  // namespace

const char* status_name(int s)
{
    switch (s) {
    case kOk: return "ok";
    case kCompile: return "compile";
    case kLaunch: return "launch";
    default: return "verify";
    }
}

int status_from(const std::string& n)
{
    if (n == "ok") return kOk;
    if (n == "compile") return kCompile;
    if (n == "launch") return kLaunch;
    return kVerify;
}

double median_of(std::vector<double> v)
{
    std::sort(v.begin(), v.end());
    const size_t n = v.size();
    if (n == 0) return 0.0;
    return (n % 2) ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

double quantile_nearest(std::vector<double> v, double p)
{
    std::sort(v.begin(), v.end());
    if (v.empty()) return 0.0;
    size_t rank = (size_t)std::ceil(p * (double)v.size());
    if (rank < 1) rank = 1;
    return v[std::min(rank, v.size()) - 1];
}

namespace {

double gflops_of(const conv2d_shape& s, double ms)
{
    return 2.0 * s.out_h * (double)s.out_w * s.filt_h * s.filt_w / (ms * 1e-3) / 1e9;
}

// ---------------------------------------------------------------- measurers

class Measurer : public MeasurerT<conv2d_config> {
public:
    virtual int lds_limit() const = 0;
};

class SyntheticMeasurer : public Measurer {
public:
    SyntheticMeasurer(conv2d_cost_fn fn, void* user) : fn_(fn), user_(user) {}
    std::string arch() const override { return "synthetic"; }
    int lds_limit() const override { return kLdsLimitGfx950; }
    int prepare(const std::vector<conv2d_config>& cfgs, std::vector<int>* status, double* seconds) override
    {
        status->assign(cfgs.size(), kOk);
        for (size_t i = 0; i < cfgs.size(); ++i) {
            double v = fn_(&cfgs[i], user_);
            if (v == (double)CONV2D_ECOMPILE) (*status)[i] = kCompile;
        }
        *seconds = 0;
        return CONV2D_OK;
    }
    int measure(const conv2d_config& c, int, int reps, double, Record* r) override
    {
        double v = fn_(&c, user_);
        r->c = c;
        if (v < 0) {
            r->status = (v == (double)CONV2D_ELAUNCH) ? kLaunch
                        : (v == (double)CONV2D_ECOMPILE) ? kCompile : kVerify;
            return CONV2D_OK;
        }
        r->status = kOk;
        r->ms = r->ms_min = r->ms_p90 = v;
        r->reps = reps;
        return CONV2D_OK;
    }

private:
    conv2d_cost_fn fn_;
    void* user_;
};

class GpuMeasurer : public Measurer {
public:
    GpuMeasurer(const conv2d_shape& s, const conv2d_tune_opts& o) : s_(s), o_(o) {}
    ~GpuMeasurer() override
    {
        if (stream_) hipStreamSynchronize(stream_);
        for (float* p : {d_in_, d_f_, d_out_, d_ref_, d_flush_})
            if (p) hipFree(p);
        for (size_t k = 1; k < in_sets_.size(); ++k) {
            hipFree(in_sets_[k]);
            hipFree(out_sets_[k]);
        }
        if (d_count_) hipFree(d_count_);
        if (e0_) hipEventDestroy(e0_);
        if (e1_) hipEventDestroy(e1_);
        if (stream_) hipStreamDestroy(stream_);
    }
    std::string arch() const override { return dev_.arch; }
    int lds_limit() const override { return dev_.lds_limit; }

    int init()
    {
        int rc = current_device_info(&dev_);
        if (rc) return rc;
        P_ = (size_t)s_.out_w + s_.filt_w - 1;
        n_in_ = ((size_t)s_.out_h + s_.filt_h - 1) * P_;
        n_out_ = (size_t)s_.out_h * s_.out_w;
        vin_ = vout_ = kVec;
        CONV2D_HIP(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
        CONV2D_HIP(hipEventCreate(&e0_));
        CONV2D_HIP(hipEventCreate(&e1_));
        if (hipMalloc(&d_in_, n_in_ * 4) != hipSuccess || hipMalloc(&d_f_, 4ull * s_.filt_h * s_.filt_w) != hipSuccess ||
            hipMalloc(&d_out_, n_out_ * 4) != hipSuccess || hipMalloc(&d_ref_, n_out_ * 4) != hipSuccess ||
            hipMalloc(&d_count_, sizeof(unsigned)) != hipSuccess)
            return fail(CONV2D_ENOMEM, "tuner: device allocation failed");
        if (o_.flush_mall) {
            n_flush_ = (512ull << 20) / 4;
            if (hipMalloc(&d_flush_, n_flush_ * 4) != hipSuccess)
                return fail(CONV2D_ENOMEM, "tuner: flush buffer allocation failed");
            rc = launch_fill_value(d_flush_, n_flush_, 0.0f, stream_);  // the flush reads zeros
            if (rc) return rc;
        }
        rc = launch_fill_uniform(d_in_, n_in_, 1, 0, stream_);
        if (!rc) rc = launch_fill_uniform(d_f_, (size_t)s_.filt_h * s_.filt_w, 2, 0, stream_);
        if (!rc) rc = launch_reference(s_, d_in_, d_f_, d_ref_, stream_);
        if (rc) return rc;
        // Copies of input and output for sustained timing: together at least
        // 512 MiB (twice the last-level cache), at most 8 sets.
        const size_t set_bytes = 4 * (n_in_ + n_out_);
        const size_t n_sets = std::min<size_t>(8, std::max<size_t>(1, ((512ull << 20) + set_bytes - 1) / set_bytes));
        in_sets_.assign(1, d_in_);
        out_sets_.assign(1, d_out_);
        for (size_t k = 1; k < n_sets; ++k) {
            float *a = nullptr, *b = nullptr;
            if (hipMalloc(&a, n_in_ * 4) != hipSuccess) return fail(CONV2D_ENOMEM, "tuner: device allocation failed");
            if (hipMalloc(&b, n_out_ * 4) != hipSuccess) {
                hipFree(a);
                return fail(CONV2D_ENOMEM, "tuner: device allocation failed");
            }
            in_sets_.push_back(a);
            out_sets_.push_back(b);
            rc = launch_fill_uniform(a, n_in_, 1, 0, stream_);
            if (rc) return rc;
        }
        CONV2D_HIP(hipStreamSynchronize(stream_));
        return CONV2D_OK;
    }

    void set_sustained(bool on) override { sustained_ = on; }

    int prepare(const std::vector<conv2d_config>& cfgs, std::vector<int>* status, double* seconds) override
    {
        const double t0 = now_s();
        status->assign(cfgs.size(), kOk);
        code_.assign(cfgs.size(), {});
        index_.clear();
        for (size_t i = 0; i < cfgs.size(); ++i) index_[config_str(cfgs[i])] = i;
        int nthreads = o_.threads > 0 ? o_.threads : (int)std::thread::hardware_concurrency();
        nthreads = std::max(1, std::min(nthreads, 16));
        std::atomic<size_t> next{0}, compiled{0};
        std::vector<std::thread> pool;
        for (int t = 0; t < nthreads; ++t)
            pool.emplace_back([&] {
                for (;;) {
                    size_t i = next++;
                    if (i >= cfgs.size()) break;
                    if (compile_direct(s_, cfgs[i], vin_, vout_, dev_.arch, &code_[i], nullptr) != CONV2D_OK)
                        (*status)[i] = kCompile;
                    const size_t done_n = ++compiled;
                    if (o_.verbose && done_n % 200 == 0)
                        std::fprintf(stderr, "[tune] compiled %zu/%zu\n", done_n, cfgs.size());
                }
            });
        for (auto& th : pool) th.join();
        *seconds = now_s() - t0;
        if (o_.verbose)
            std::fprintf(stderr, "[tune] compiled %zu configurations in %.1f s\n", cfgs.size(), *seconds);
        return CONV2D_OK;
    }

    int measure(const conv2d_config& c, int warmup, int reps, double best_so_far, Record* r) override
    {
        r->c = c;
        auto it = index_.find(config_str(c));
        if (it == index_.end()) return fail(CONV2D_EINVAL, "config not prepared");
        std::vector<char>& code = code_[it->second];
        Module m;
        if (load_module(code, direct_kernel_name(s_, c), &m) != CONV2D_OK) { r->status = kLaunch; return CONV2D_OK; }
        std::vector<char>().swap(code);
        int rc = run_checked(m, c, r);
        if (rc == CONV2D_OK && r->status == kOk) rc = time_it(m, c, warmup, reps, best_so_far, r);
        unload_module(&m);
        return rc;
    }

private:
    // What conv2d_run enqueues: the filter copy into the module's constant
    // array (filter_in_const = 1), then the kernel. The tuner times exactly
    // this, so a constant-memory filter is charged for its copy.
    int launch(const Module& m, const conv2d_config& c, size_t set = 0)
    {
        if (c.filter_in_const) {
            if (!m.const_filter) return fail(CONV2D_ELAUNCH, "module has no conv_filter symbol");
            if (hipMemcpyAsync(m.const_filter, d_f_, 4ull * s_.filt_h * s_.filt_w, hipMemcpyDeviceToDevice,
                               stream_) != hipSuccess)
                return fail(CONV2D_ELAUNCH, "filter copy failed");
        }
        return launch_direct(m, s_, c, in_sets_[set], d_f_, out_sets_[set], stream_);
    }

    // One launch on a NaN-filled output, then a bitwise comparison.
    int run_checked(const Module& m, const conv2d_config& c, Record* r)
    {
        int rc = launch_fill_value(d_out_, n_out_, __builtin_nanf(""), stream_);
        if (rc) return rc;
        if (launch(m, c) != CONV2D_OK) {
            (void)hipGetLastError();
            r->status = kLaunch;
            return CONV2D_OK;
        }
        hipError_t e = hipStreamSynchronize(stream_);
        if (e != hipSuccess) return hip_fail(e, "tuner: kernel execution");
        CONV2D_HIP(hipMemsetAsync(d_count_, 0, sizeof(unsigned), stream_));
        rc = launch_count_mismatch(d_out_, d_ref_, n_out_, d_count_, stream_);
        if (rc) return rc;
        unsigned bad = 0;
        CONV2D_HIP(hipMemcpyAsync(&bad, d_count_, sizeof bad, hipMemcpyDeviceToHost, stream_));
        CONV2D_HIP(hipStreamSynchronize(stream_));
        r->status = bad ? kVerify : kOk;
        return CONV2D_OK;
    }

    int time_it(const Module& m, const conv2d_config& c, int warmup, int reps, double best_so_far, Record* r)
    {
        if (sustained_) {
            const size_t n = in_sets_.size();
            for (int k = 0; k < warmup + (int)n; ++k)
                if (launch(m, c, (size_t)k % n)) return fail(CONV2D_ELAUNCH, "tuner: warm-up launch failed");
            CONV2D_HIP(hipEventRecord(e0_, stream_));
            for (int k = 0; k < reps; ++k)
                if (launch(m, c, (size_t)k % n)) return fail(CONV2D_ELAUNCH, "tuner: timed launch failed");
            CONV2D_HIP(hipEventRecord(e1_, stream_));
            CONV2D_HIP(hipEventSynchronize(e1_));
            float ms = 0;
            CONV2D_HIP(hipEventElapsedTime(&ms, e0_, e1_));
            r->ms = r->ms_min = r->ms_p90 = ms / reps;
            r->reps = reps;
            return CONV2D_OK;
        }
        for (int k = 0; k < warmup; ++k)
            if (launch(m, c)) return fail(CONV2D_ELAUNCH, "tuner: warm-up launch failed");
        std::vector<double> t;
        for (int k = 0; k < reps; ++k) {
            if (d_flush_ && launch_flush(d_flush_, n_flush_, stream_)) return CONV2D_ELAUNCH;
            CONV2D_HIP(hipEventRecord(e0_, stream_));
            if (launch(m, c)) return fail(CONV2D_ELAUNCH, "tuner: timed launch failed");
            CONV2D_HIP(hipEventRecord(e1_, stream_));
            CONV2D_HIP(hipEventSynchronize(e1_));
            float ms = 0;
            CONV2D_HIP(hipEventElapsedTime(&ms, e0_, e1_));
            t.push_back(ms);
            // Far slower than the best so far: three samples are enough.
            if (best_so_far > 0 && k >= 2 && t[0] > 20.0 * best_so_far) break;
        }
        r->ms = median_of(t);
        r->ms_min = *std::min_element(t.begin(), t.end());
        r->ms_p90 = quantile_nearest(t, 0.9);
        r->reps = (int)t.size();
        return CONV2D_OK;
    }

    conv2d_shape s_;
    conv2d_tune_opts o_;
    DeviceInfo dev_;
    size_t P_ = 0, n_in_ = 0, n_out_ = 0, n_flush_ = 0;
    int vin_ = 1, vout_ = 1;
    float *d_in_ = nullptr, *d_f_ = nullptr, *d_out_ = nullptr, *d_ref_ = nullptr, *d_flush_ = nullptr;
    unsigned* d_count_ = nullptr;
    hipStream_t stream_ = nullptr;
    hipEvent_t e0_ = nullptr, e1_ = nullptr;
    std::vector<std::vector<char>> code_;
    std::map<std::string, size_t> index_;
    std::vector<float*> in_sets_, out_sets_;   // set 0 is d_in_ / d_out_
    bool sustained_ = false;
};

// ---------------------------------------------------------------- the search

std::string result_line(const std::string& arch, const conv2d_shape& s, const Record& r)
{
    char b[640];
    std::snprintf(b, sizeof b,
                  "{\"arch\":\"%s\",\"src\":\"%s\",\"shape\":%s,\"config\":%s,\"status\":\"%s\","
                  "\"ms\":%.6f,\"ms_min\":%.6f,\"ms_p90\":%.6f,\"reps\":%d,\"gflops\":%.3f}",
                  json_escape(arch).c_str(), hex64(direct_source_hash()).c_str(), shape_json(s).c_str(),
                  config_json(r.c).c_str(), status_name(r.status), r.ms, r.ms_min, r.ms_p90, r.reps,
                  r.status == kOk && r.ms > 0 ? gflops_of(s, r.ms) : 0.0);
    return b;
}

void load_results(const std::string& path, const std::string& arch, const conv2d_shape& s,
                  std::map<std::string, Record>* out)
{
    std::ifstream f(path);
    if (!f) return;
    const std::string src = hex64(direct_source_hash());
    std::string line;
    while (std::getline(f, line)) {
        JsonObj o;
        if (!json_parse_line(line, &o)) continue;
        if (o.str["arch"] != arch || o.str["src"] != src || !json_shape_is(o, s)) continue;
        Record r;
        if (!json_config(o, &r.c)) continue;
        r.status = status_from(o.str["status"]);
        r.ms = o.num["ms"];
        r.ms_min = o.num["ms_min"];
        r.ms_p90 = o.num["ms_p90"];
        r.reps = (int)o.num["reps"];
        (*out)[config_str(r.c)] = r;
    }
}

// SplitMix64 output number k of stream `seed` (Steele, Lea and Flood 2014).
uint64_t splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Random-restart hill climbing over the legal points (a local-search
// strategy in place of brute force, for shapes where a full sweep costs too
// much). From a start point, all not-yet-evaluated neighbours (one parameter
// moved one step along its ordered value list) are evaluated and the walk
// moves to the fastest neighbour while that improves; at a local minimum it
// restarts from the idx-th not-yet-evaluated point in enumeration order, with
// idx = splitmix64(seed, restart) mod (number not yet evaluated). Stops after
// max_evals evaluations (failures count). Ties go to the smallest tuple.
int local_search(const conv2d_shape& s, const conv2d_tune_opts& o, Measurer* meas, conv2d_tune_result* res,
                 const std::vector<conv2d_config>& legal)
{
    const double t0 = now_s();
    std::map<std::string, int> index;
    for (size_t i = 0; i < legal.size(); ++i) index[config_str(legal[i])] = (int)i;
    std::vector<int> state(legal.size(), 0);  // 0 not evaluated, 1 ok, -1 failed
    std::vector<double> ms(legal.size(), 0.0);
    int evals = 0;
    const int budget = o.max_evals > 0 ? o.max_evals : 100;

    auto evaluate = [&](const std::vector<int>& ids) -> int {
        std::vector<conv2d_config> cfgs;
        for (int i : ids) cfgs.push_back(legal[i]);
        std::vector<int> st;
        double sec = 0;
        int rc = meas->prepare(cfgs, &st, &sec);
        if (rc) return rc;
        res->compile_s += sec;
        for (size_t k = 0; k < ids.size() && evals < budget; ++k) {
            const int i = ids[k];
            Record r;
            r.c = legal[i];
            if (st[k] != kOk) r.status = st[k];
            else {
                rc = meas->measure(legal[i], o.warmup, o.reps, 0, &r);
                if (rc) return rc;
            }
            ++evals;
            state[i] = r.status == kOk ? 1 : -1;
            ms[i] = r.ms;
            if (r.status == kCompile) res->n_compile_fail++;
            else if (r.status == kLaunch) res->n_launch_fail++;
            else if (r.status == kVerify) res->n_verify_fail++;
            if (o.results_path && *o.results_path) append_line(o.results_path, result_line(meas->arch(), s, r));
        }
        return CONV2D_OK;
    };
    auto neighbours = [&](int i) {
        static const std::vector<std::vector<int>> axes = {
            {16, 32, 64, 128}, {1, 2, 4, 8, 16}, {1, 2, 4, 8}, {1, 2, 4, 8}, {0, 1}, {0, 1}};
        std::vector<int> out;
        const conv2d_config& c = legal[i];
        int v[6] = {c.block_x, c.block_y, c.tile_x, c.tile_y, c.use_lds, c.filter_in_const};
        for (int k = 0; k < 6; ++k) {
            const auto& vals = axes[k];
            const int pos = (int)(std::find(vals.begin(), vals.end(), v[k]) - vals.begin());
            for (int q : {pos - 1, pos + 1}) {
                if (q < 0 || q >= (int)vals.size()) continue;
                int w[6];
                std::copy(v, v + 6, w);
                w[k] = vals[q];
                conv2d_config n{w[0], w[1], w[2], w[3], w[4], w[5], c.unroll};
                auto it = index.find(config_str(n));
                if (it != index.end()) out.push_back(it->second);
            }
        }
        return out;
    };
    auto better = [&](int a, int b) {  // a strictly preferable to b
        return ms[a] < ms[b] || (ms[a] == ms[b] && config_less(legal[a], legal[b]));
    };

    uint64_t restart = 0;
    while (evals < budget) {
        std::vector<int> fresh;
        for (size_t i = 0; i < legal.size(); ++i)
            if (!state[i]) fresh.push_back((int)i);
        if (fresh.empty()) break;
        int cur = fresh[splitmix64((uint64_t)o.seed, restart++) % fresh.size()];
        int rc = evaluate({cur});
        if (rc) return rc;
        if (state[cur] != 1) continue;
        while (evals < budget) {
            std::vector<int> todo;
            const std::vector<int> nb = neighbours(cur);
            for (int n : nb)
                if (!state[n]) todo.push_back(n);
            rc = evaluate(todo);
            if (rc) return rc;
            int next = -1;
            for (int n : nb)
                if (state[n] == 1 && (next < 0 || better(n, next))) next = n;
            if (next < 0 || !(ms[next] < ms[cur])) break;
            cur = next;
        }
    }
    int best = -1;
    for (size_t i = 0; i < legal.size(); ++i)
        if (state[i] == 1 && (best < 0 || better((int)i, best))) best = (int)i;
    res->n_timed = 0;
    for (int st : state) res->n_timed += (st == 1);
    res->measure_s = now_s() - t0;
    if (best < 0) return fail(CONV2D_EVERIFY, "local search: no configuration compiled, ran and verified");
    res->best = legal[best];
    res->best_ms = ms[best];
    res->best_gflops = gflops_of(s, ms[best]);
    res->evaluations = evals;
    if (o.winners_path && *o.winners_path) {
        int rc = cache_store(o.winners_path, meas->arch(), s, legal[best], ms[best]);
        if (rc) return rc;
    }
    return CONV2D_OK;
}

int tune_core(const conv2d_shape& s, const conv2d_tune_opts& o, Measurer* meas, conv2d_tune_result* res)
{
    *res = conv2d_tune_result{};
    const int n_space = conv2d_space(s, o.unroll, -1, nullptr, 0);
    if (n_space < 0) return n_space;
    std::vector<conv2d_config> space(n_space);
    conv2d_space(s, o.unroll, -1, space.data(), n_space);
    res->n_space = n_space;

    conv2d_config dflt;
    conv2d_default_config(&dflt);
    bool default_in_space = false;
    std::vector<conv2d_config> legal;
    for (const auto& c : space) {
        if (conv2d_config_check(s, &c, meas->lds_limit()) != CONV2D_OK) { res->n_illegal++; continue; }
        legal.push_back(c);
        if (config_equal(c, dflt)) default_in_space = true;
    }
    clear_error();
    if (o.max_configs > 0 && (int)legal.size() > o.max_configs) legal.resize(o.max_configs);
    if (o.strategy == 1) return local_search(s, o, meas, res, legal);
    std::vector<conv2d_config> candidates = legal;
    if (!default_in_space && conv2d_config_check(s, &dflt, meas->lds_limit()) == CONV2D_OK)
        candidates.push_back(dflt);  // timed for tuned/default, not eligible as winner
    clear_error();

    std::map<std::string, Record> done;
    if (o.results_path && *o.results_path) load_results(o.results_path, meas->arch(), s, &done);
    std::vector<conv2d_config> todo;
    for (const auto& c : candidates)
        if (!done.count(config_str(c))) todo.push_back(c);
    res->n_resumed = (int)(candidates.size() - todo.size());

    const double t0 = now_s();
    double best = 0;
    for (const auto& kv : done)
        if (kv.second.status == kOk && (best == 0 || kv.second.ms < best)) best = kv.second.ms;
    auto key = [](const conv2d_config& c) { return config_str(c); };
    auto sink = [&](const Record& r) {
        if (o.results_path && *o.results_path) append_line(o.results_path, result_line(meas->arch(), s, r));
    };
    int rc = measure_all(todo, meas, o.warmup, o.reps, o.verbose != 0, key, sink, &done, &best, &res->compile_s);
    if (rc) return rc;

    // Optional refinement: the ten fastest points again with every other
    // unroll value (the partial-unroll factor the paper makes tunable).
    if (o.refine_unroll) {
        std::vector<Record> ok;
        for (const auto& c : legal) {
            const Record& r = done[config_str(c)];
            if (r.status == kOk) ok.push_back(r);
        }
        std::sort(ok.begin(), ok.end(), [](const Record& a, const Record& b) { return a.ms < b.ms; });
        if (ok.size() > 10) ok.resize(10);
        std::vector<conv2d_config> extra;
        for (const auto& r : ok)
            for (int u : {0, 1, 2, 4}) {
                conv2d_config c2 = r.c;
                c2.unroll = u;
                if (u == r.c.unroll || conv2d_config_check(s, &c2, meas->lds_limit()) != CONV2D_OK) continue;
                bool seen = false;
                for (const auto& e : extra) seen = seen || config_equal(e, c2);
                if (!seen) extra.push_back(c2);
            }
        clear_error();
        std::vector<conv2d_config> todo2;
        for (const auto& c : extra)
            if (!done.count(config_str(c))) todo2.push_back(c);
        rc = measure_all(todo2, meas, o.warmup, o.reps, false, key, sink, &done, &best, &res->compile_s);
        if (rc) return rc;
        for (const auto& c : extra) {
            legal.push_back(c);
            candidates.push_back(c);
        }
        if (o.verbose) std::fprintf(stderr, "[tune] refined %zu unroll variants\n", extra.size());
    }

    // Collect the timed points among the candidates.
    std::vector<Record> timed;
    for (const auto& c : candidates) {
        const Record& r = done[config_str(c)];
        if (r.status == kCompile) res->n_compile_fail++;
        else if (r.status == kLaunch) res->n_launch_fail++;
        else if (r.status == kVerify) res->n_verify_fail++;
        else timed.push_back(r);
    }
    std::set<std::string> legal_keys;
    for (const auto& c : legal) legal_keys.insert(config_str(c));
    std::vector<Record> eligible;
    for (const auto& r : timed)
        if (legal_keys.count(config_str(r.c))) eligible.push_back(r);
    res->n_timed = (int)eligible.size();
    if (eligible.empty()) return fail(CONV2D_EVERIFY, "no configuration compiled, ran and verified");

    // Re-time the ten fastest with sustained launches; the winner is the
    // lowest sustained time, ties within tie_rel going to the smallest tuple.
    Record win;
    std::vector<Record> top;
    rc = retime_and_pick(&eligible, meas, o.warmup, o.retime_reps, 10, o.tie_rel, config_less, &top, &win);
    if (rc) return rc;
    res->measure_s = now_s() - t0 - res->compile_s;
    res->evaluations = (int)(candidates.size()) - res->n_resumed;
    res->best = win.c;
    res->best_ms = win.ms;
    for (int k = 0; k < 5 && k < (int)top.size(); ++k) {
        res->top[k] = top[k].c;
        res->top_ms[k] = top[k].ms;
    }

    // Tuning impact: maximum over median throughput across the space.
    std::vector<double> perf;
    for (const auto& r : eligible) perf.push_back(gflops_of(s, r.ms));
    const double med_perf = median_of(perf);
    const double max_perf = *std::max_element(perf.begin(), perf.end());
    res->median_gflops = med_perf;
    res->median_ms = 2.0 * s.out_h * (double)s.out_w * s.filt_h * s.filt_w / (med_perf * 1e9) * 1e3;
    res->best_gflops = gflops_of(s, win.ms);
    res->impact = max_perf / med_perf;   // both from the sweep's timing

    {
        const auto wit = done.find(config_str(win.c));
        if (wit != done.end() && wit->second.status == kOk) res->best_sweep_ms = wit->second.ms;
    }

    // The default configuration's rank in the sweep, and its time in the
    // winner's timing mode (tuned/default compares like with like: the
    // sustained re-timing favours large launches less than flushed single
    // launches do, most of all on small problems).
    const auto dit = done.find(config_str(dflt));
    if (dit != done.end() && dit->second.status == kOk) {
        res->default_sweep_ms = dit->second.ms;
        int faster = 0;
        for (const auto& r : eligible)
            if (r.ms < res->default_sweep_ms && !config_equal(r.c, dflt)) ++faster;
        res->default_rank = faster + 1;
        res->default_ms = res->default_sweep_ms;
        if (o.retime_reps > 0) {
            Record d;
            rc = retime_one(dflt, meas, o.warmup, o.retime_reps, &d);
            if (rc) return rc;
            res->default_ms = d.status == kOk ? d.ms : 0;
        }
        res->default_gflops = res->default_ms > 0 ? gflops_of(s, res->default_ms) : 0;
    }

    if (o.winners_path && *o.winners_path) {
        rc = cache_store(o.winners_path, meas->arch(), s, win.c, win.ms);
        if (rc) return rc;
    }
    return CONV2D_OK;
}

conv2d_tune_opts resolve(const conv2d_tune_opts* o)
{
    conv2d_tune_opts r;
    conv2d_tune_defaults(&r);
    if (o) r = *o;
    if (r.warmup < 0) r.warmup = 0;
    if (r.reps < 1) r.reps = 1;
    if (r.retime_reps < 0) r.retime_reps = 0;
    if (r.tie_rel < 0) r.tie_rel = 0;
    return r;
}

}  // namespace
}  // namespace conv2d

using namespace conv2d;

extern "C" void conv2d_tune_defaults(conv2d_tune_opts* o)
{
    if (!o) return;
    *o = conv2d_tune_opts{};
    o->warmup = 2;
    o->reps = 20;
    o->retime_reps = 200;
    o->flush_mall = 1;
    o->threads = 0;
    o->unroll = 1;
    o->max_configs = 0;
    o->tie_rel = 0.005;
    o->strategy = 0;
    o->max_evals = 100;
    o->seed = 1;
}

extern "C" int conv2d_tune(conv2d_shape s, const conv2d_tune_opts* opts, conv2d_tune_result* res)
{
    clear_error();
    if (!res) return fail(CONV2D_EINVAL, "res is NULL");
    int rc = shape_check(s);
    if (rc) return rc;
    conv2d_tune_opts o = resolve(opts);
    std::string why;
    conv2d_config probe{16, 1, 1, 1, 0, 0, o.unroll};
    if (!config_axes_valid(probe, &why)) return fail(CONV2D_EINVAL, why);
    GpuMeasurer m(s, o);
    rc = m.init();
    if (rc) return rc;
    return tune_core(s, o, &m, res);
}

extern "C" int conv2d_tune_synthetic(conv2d_shape s, conv2d_cost_fn cost, void* user,
                                     const conv2d_tune_opts* opts, conv2d_tune_result* res)
{
    clear_error();
    if (!res || !cost) return fail(CONV2D_EINVAL, "cost and res must be non-NULL");
    int rc = shape_check(s);
    if (rc) return rc;
    conv2d_tune_opts o = resolve(opts);
    SyntheticMeasurer m(cost, user);
    return tune_core(s, o, &m, res);
}

extern "C" int conv2d_cache_lookup(const char* path, const char* arch, conv2d_shape s, conv2d_config* cfg,
                                   double* ms)
{
    clear_error();
    std::string a;
    if (arch) a = arch;
    else {
        DeviceInfo d;
        int rc = current_device_info(&d);
        if (rc) return rc;
        a = d.arch;
    }
    return cache_lookup(path ? path : winners_default_path(), a, s, cfg, ms);
}

extern "C" int conv2d_cache_store(const char* path, const char* arch, conv2d_shape s, const conv2d_config* cfg,
                                  double ms)
{
    clear_error();
    if (!cfg) return fail(CONV2D_EINVAL, "cfg is NULL");
    std::string a;
    if (arch) a = arch;
    else {
        DeviceInfo d;
        int rc = current_device_info(&d);
        if (rc) return rc;
        a = d.arch;
    }
    return cache_store(path ? path : winners_default_path(), a, s, *cfg, ms);
}

extern "C" int conv2d_benchmark(conv2d_shape s, const conv2d_config* cfg, int warmup, int reps, int flush_mall,
                                double* median_ms, double* min_ms)
{
    clear_error();
    if (!cfg) return fail(CONV2D_EINVAL, "cfg is NULL");
    int rc = shape_check(s);
    if (rc) return rc;
    conv2d_tune_opts o;
    conv2d_tune_defaults(&o);
    o.flush_mall = flush_mall ? 1 : 0;
    o.threads = 1;
    GpuMeasurer m(s, o);
    rc = m.init();
    if (rc) return rc;
    rc = conv2d_config_check(s, cfg, m.lds_limit());
    if (rc) return rc;
    std::vector<int> st;
    double sec = 0;
    rc = m.prepare({*cfg}, &st, &sec);
    if (rc) return rc;
    if (st[0] != kOk) return CONV2D_ECOMPILE;  // message left by the compiler
    Record r;
    rc = m.measure(*cfg, warmup < 0 ? 0 : warmup, reps < 1 ? 1 : reps, 0, &r);
    if (rc) return rc;
    if (r.status == kLaunch) return fail(CONV2D_ELAUNCH, "benchmark: launch failed");
    if (r.status == kVerify) return fail(CONV2D_EVERIFY, "benchmark: output differs from the reference kernel");
    if (median_ms) *median_ms = r.ms;
    if (min_ms) *min_ms = r.ms_min;
    return CONV2D_OK;
}
