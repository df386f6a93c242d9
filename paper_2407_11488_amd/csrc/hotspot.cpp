// Hotspot stencil host side: configuration legality and space, run-time
// compilation of hotspot.hip, plans and runs (temporal tiling over several
// launches), the one-step-per-launch reference, and the tuner, which runs on
// the same search machinery as the convolution tuner (search.h).
#include <algorithm>
#include <array>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <memory>
#include <set>
#include <thread>

#include "hotspot.h"
#include "internal.h"
#include "search.h"

namespace conv2d {
namespace {

#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wc23-extensions"
const char kHotspotSource[] = {
#embed "hotspot.hip"
    , 0};
#pragma clang diagnostic pop

const std::string& hs_source()
{
    static const std::string s(kHotspotSource);
    return s;
}

uint64_t hs_source_hash()
{
    static const uint64_t h = fnv1a(code_text(hs_source()));
    return h;
}

// The axes of the space, each in ascending order.
const std::vector<int> kBlockX = {16, 32, 64, 128, 256};
const std::vector<int> kBlockY = {1, 2, 4, 8, 16};
const std::vector<int> kTile = {1, 2, 4};
const std::vector<int> kTemporal = {1, 2, 3, 4, 6, 8};
const std::vector<int> kUnrollT = {0, 1};
const std::vector<int> kShPower = {0, 1};

bool on_axis(int v, const std::vector<int>& axis) { return std::find(axis.begin(), axis.end(), v) != axis.end(); }

int values(const hotspot_config& c, int k)
{
    const int v[7] = {c.block_x, c.block_y, c.tile_x, c.tile_y, c.temporal, c.unroll_t, c.sh_power};
    return v[k];
}

std::string hs_str(const hotspot_config& c)
{
    char b[96];
    std::snprintf(b, sizeof b, "%d,%d,%d,%d,%d,%d,%d", c.block_x, c.block_y, c.tile_x, c.tile_y, c.temporal,
                  c.unroll_t, c.sh_power);
    return b;
}

bool hs_less(const hotspot_config& a, const hotspot_config& b)
{
    for (int k = 0; k < 7; ++k)
        if (values(a, k) != values(b, k)) return values(a, k) < values(b, k);
    return false;
}

bool hs_equal(const hotspot_config& a, const hotspot_config& b) { return !hs_less(a, b) && !hs_less(b, a); }

std::string hs_kernel_name(const hotspot_config& c)
{
    char b[96];
    std::snprintf(b, sizeof b, "hotspot_b%dx%d_t%dx%d_tt%du%dp%d", c.block_x, c.block_y, c.tile_x, c.tile_y,
                  c.temporal, c.unroll_t, c.sh_power);
    return b;
}

std::vector<std::string> hs_options(const hotspot_config& c, const std::string& arch)
{
    auto D = [](const char* k, int v) { return std::string("-D") + k + "=" + std::to_string(v); };
    return {
        "--offload-arch=" + arch,
        "-O3",
        "-std=c++17",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        D("HS_BX", c.block_x), D("HS_BY", c.block_y), D("HS_TX", c.tile_x), D("HS_TY", c.tile_y),
        D("HS_TT", c.temporal), D("HS_UNROLL_T", c.unroll_t), D("HS_SH_POWER", c.sh_power),
        "-DHS_NAME=" + hs_kernel_name(c),
    };
}

int hs_compile(const hotspot_config& c, const std::string& arch, std::vector<char>* code, std::string* path)
{
    return compile_program(hs_source(), "hotspot.hip", hs_options(c, arch), "hotspot config " + hs_str(c), code,
                           path);
}

int region_rows(const hotspot_config& c) { return c.block_y * c.tile_y; }
int region_cols(const hotspot_config& c) { return c.block_x * c.tile_x; }

struct HsGeometry {
    int tiles_x = 0, tiles_y = 0, n_tiles = 0;
};

HsGeometry hs_geometry(const hotspot_shape& s, const hotspot_config& c)
{
    const int oh = region_rows(c) - 2 * c.temporal, ow = region_cols(c) - 2 * c.temporal;
    HsGeometry g;
    g.tiles_x = (s.cols + ow - 1) / ow;
    g.tiles_y = (s.rows + oh - 1) / oh;
    const long long n = (long long)g.tiles_x * g.tiles_y;
    g.n_tiles = n > INT_MAX ? -1 : (int)n;
    return g;
}

int shape_ok(const hotspot_shape& s)
{
    if (s.rows < 1 || s.cols < 1) return fail(CONV2D_EINVAL, "hotspot grid sides must be >= 1");
    return CONV2D_OK;
}

// One launch of up to c.temporal steps from tin to tout.
int hs_launch(const Module& m, const hotspot_config& c, const hotspot_shape& s, const float* tin, const float* power,
              float* tout, int steps, const hotspot_coeffs& k, hipStream_t st)
{
    const HsGeometry g = hs_geometry(s, c);
    if (g.n_tiles < 1) return fail(CONV2D_EINVAL, "hotspot: too many tiles for one launch");
    int rows = s.rows, cols = s.cols, tiles_x = g.tiles_x, n_tiles = g.n_tiles;
    hs_terms t = hs_fold(k);
    const void* a_in = tin;
    const void* a_pw = power;
    void* a_out = tout;
    void* args[] = {&a_in, &a_pw, &a_out, &rows, &cols, &steps, &tiles_x, &n_tiles, &t.ka, &t.ky, &t.kx, &t.cc, &t.q};
    hipError_t e = hipModuleLaunchKernel(m.fn, (unsigned)n_tiles, 1, 1, (unsigned)(c.block_x * c.block_y), 1, 1, 0,
                                         st, args, nullptr);
    if (e != hipSuccess) return fail(CONV2D_ELAUNCH, std::string("hotspot launch: ") + hipGetErrorString(e));
    return CONV2D_OK;
}

// The destinations of n launches ending in d_out: launch i writes d_out when
// n - 1 - i is even, d_work otherwise; it reads the previous destination
// (d_temp for the first).
template <class Launch>
int ping_pong(int n, const float* d_temp, float* d_out, float* d_work, Launch launch)
{
    const float* src = d_temp;
    for (int i = 0; i < n; ++i) {
        float* dst = ((n - 1 - i) % 2 == 0) ? d_out : d_work;
        int rc = launch(i, src, dst);
        if (rc) return rc;
        src = dst;
    }
    return CONV2D_OK;
}

bool overlaps(const void* a, size_t an, const void* b, size_t bn)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bn && y < x + an;
}

int check_buffers(const hotspot_shape& s, const float* d_temp, const float* d_power, float* d_out, float* d_work,
                  int launches)
{
    const size_t bytes = 4ull * (size_t)s.rows * (size_t)s.cols;
    int rc = check_device_range(d_temp, bytes, "d_temp");
    if (!rc) rc = check_device_range(d_power, bytes, "d_power");
    if (!rc) rc = check_device_range(d_out, bytes, "d_out");
    if (rc) return rc;
    if (overlaps(d_out, bytes, d_temp, bytes) || overlaps(d_out, bytes, d_power, bytes))
        return fail(CONV2D_EINVAL, "d_out overlaps an input");
    if (launches > 1) {
        if (!d_work) return fail(CONV2D_EINVAL, "d_work is needed when the run takes more than one launch");
        rc = check_device_range(d_work, bytes, "d_work");
        if (rc) return rc;
        if (overlaps(d_work, bytes, d_temp, bytes) || overlaps(d_work, bytes, d_power, bytes) ||
            overlaps(d_work, bytes, d_out, bytes))
            return fail(CONV2D_EINVAL, "d_work overlaps another buffer");
    }
    return CONV2D_OK;
}

int hs_run(const Module& m, const hotspot_config& c, const hotspot_shape& s, const float* d_temp,
           const float* d_power, float* d_out, float* d_work, int steps, const hotspot_coeffs& k, hipStream_t st)
{
    if (steps == 0) {
        CONV2D_HIP(hipMemcpyAsync(d_out, d_temp, 4ull * (size_t)s.rows * (size_t)s.cols, hipMemcpyDeviceToDevice, st));
        return CONV2D_OK;
    }
    const int n = (steps + c.temporal - 1) / c.temporal;
    return ping_pong(n, d_temp, d_out, d_work, [&](int i, const float* src, float* dst) {
        const int this_steps = std::min(c.temporal, steps - i * c.temporal);
        return hs_launch(m, c, s, src, d_power, dst, this_steps, k, st);
    });
}

// ---------------------------------------------------------------- winners cache

std::string hs_winners_default_path() { return library_dir() + "/tuned/hotspot_winners.jsonl"; }

bool json_hs_config(const JsonObj& o, hotspot_config* c)
{
    auto it = o.arr.find("config");
    if (it == o.arr.end() || it->second.size() != 7) return false;
    const auto& a = it->second;
    *c = hotspot_config{(int)a[0], (int)a[1], (int)a[2], (int)a[3], (int)a[4], (int)a[5], (int)a[6]};
    return true;
}

bool json_grid_is(const JsonObj& o, const hotspot_shape& s)
{
    auto it = o.arr.find("shape");
    return it != o.arr.end() && it->second.size() == 2 && (int)it->second[0] == s.rows &&
           (int)it->second[1] == s.cols;
}

// The winner for a grid size: an entry for the current kernel source, else
// one for an older source.
int hs_cache_lookup(const std::string& path, const std::string& arch, const hotspot_shape& s, hotspot_config* c,
                    bool* stale)
{
    std::ifstream f(path);
    if (!f) return fail(CONV2D_ENOTUNED, "no hotspot winners cache at " + path);
    const std::string src = hex64(hs_source_hash());
    bool have_cur = false, have_old = false;
    hotspot_config cur{}, old{};
    std::string line;
    while (std::getline(f, line)) {
        JsonObj o;
        if (!json_parse_line(line, &o) || o.str["arch"] != arch || !json_grid_is(o, s)) continue;
        hotspot_config cc;
        if (!json_hs_config(o, &cc)) continue;
        if (o.str["src"] == src) { cur = cc; have_cur = true; }
        else { old = cc; have_old = true; }
    }
    if (!have_cur && !have_old) return fail(CONV2D_ENOTUNED, "grid size not in the hotspot winners cache");
    *c = have_cur ? cur : old;
    if (stale) *stale = !have_cur;
    return CONV2D_OK;
}

// The winner for another grid, for a grid without an entry of its own: the
// 4096 x 4096 entry first, else the most recent entry (of the current kernel
// source before older ones) whose configuration is legal for grid s.
int hs_cache_lookup_other(const std::string& path, const std::string& arch, const hotspot_shape& s, int lds_limit,
                          hotspot_config* c)
{
    const hotspot_shape big{4096, 4096};
    hotspot_config cand{};
    if (hs_cache_lookup(path, arch, big, &cand, nullptr) == CONV2D_OK &&
        hotspot_config_check(s, &cand, lds_limit) == CONV2D_OK) {
        *c = cand;
        return CONV2D_OK;
    }
    std::ifstream f(path);
    if (!f) return fail(CONV2D_ENOTUNED, "no hotspot winners cache at " + path);
    const std::string src = hex64(hs_source_hash());
    bool have_cur = false, have_old = false;
    hotspot_config cur{}, old{};
    std::string line;
    while (std::getline(f, line)) {
        JsonObj o;
        if (!json_parse_line(line, &o) || o.str["arch"] != arch) continue;
        hotspot_config cc;
        if (!json_hs_config(o, &cc) || hotspot_config_check(s, &cc, lds_limit) != CONV2D_OK) continue;
        if (o.str["src"] == src) { cur = cc; have_cur = true; }
        else { old = cc; have_old = true; }
    }
    clear_error();
    if (!have_cur && !have_old) return fail(CONV2D_ENOTUNED, "no legal hotspot winner for this grid");
    *c = have_cur ? cur : old;
    return CONV2D_OK;
}

std::string record_line(const std::string& arch, const hotspot_shape& s, int steps, const RecordT<hotspot_config>& r,
                        double gflops)
{
    char b[640];
    std::snprintf(b, sizeof b,
                  "{\"arch\":\"%s\",\"src\":\"%s\",\"shape\":[%d,%d],\"steps\":%d,\"config\":[%s],\"status\":\"%s\","
                  "\"ms\":%.6f,\"ms_min\":%.6f,\"ms_p90\":%.6f,\"reps\":%d,\"gflops\":%.3f}",
                  json_escape(arch).c_str(), hex64(hs_source_hash()).c_str(), s.rows, s.cols, steps,
                  hs_str(r.c).c_str(), status_name(r.status), r.ms, r.ms_min, r.ms_p90, r.reps, gflops);
    return b;
}

double hs_flops(const hotspot_shape& s, int steps) { return 14.0 * (double)s.rows * (double)s.cols * steps; }

// ---------------------------------------------------------------- tuner

class HotspotMeasurer : public MeasurerT<hotspot_config> {
public:
    HotspotMeasurer(const hotspot_shape& s, int steps, const hotspot_tune_opts& o) : s_(s), steps_(steps), o_(o) {}
    ~HotspotMeasurer() override
    {
        if (stream_) hipStreamSynchronize(stream_);
        for (float* p : {d_temp_, d_power_, d_out_, d_work_, d_ref_, d_flush_})
            if (p) hipFree(p);
        for (size_t k = 1; k < sets_.size(); ++k)
            for (float* p : sets_[k]) hipFree(p);
        if (d_count_) hipFree(d_count_);
        if (e0_) hipEventDestroy(e0_);
        if (e1_) hipEventDestroy(e1_);
        if (stream_) hipStreamDestroy(stream_);
    }
    std::string arch() const override { return dev_.arch; }
    int lds_limit() const { return dev_.lds_limit; }

    // Seeded data (temperatures and powers from the uniform generator; the
    // coefficients keep the explicit step stable) and the reference result.
    int init()
    {
        int rc = current_device_info(&dev_);
        if (rc) return rc;
        n_ = (size_t)s_.rows * (size_t)s_.cols;
        CONV2D_HIP(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
        CONV2D_HIP(hipEventCreate(&e0_));
        CONV2D_HIP(hipEventCreate(&e1_));
        for (float** p : {&d_temp_, &d_power_, &d_out_, &d_work_, &d_ref_})
            if (hipMalloc(p, n_ * 4) != hipSuccess) return fail(CONV2D_ENOMEM, "hotspot tuner: device allocation");
        if (hipMalloc(&d_count_, sizeof(unsigned)) != hipSuccess)
            return fail(CONV2D_ENOMEM, "hotspot tuner: device allocation");
        if (o_.flush_mall) {
            n_flush_ = (512ull << 20) / 4;
            if (hipMalloc(&d_flush_, n_flush_ * 4) != hipSuccess)
                return fail(CONV2D_ENOMEM, "hotspot tuner: flush buffer allocation");
            rc = launch_fill_value(d_flush_, n_flush_, 0.0f, stream_);
            if (rc) return rc;
        }
        rc = launch_fill_uniform(d_temp_, n_, 11, 0, stream_);
        if (!rc) rc = launch_fill_uniform(d_power_, n_, 12, 0, stream_);
        if (rc) return rc;
        k_ = hotspot_coeffs{0.2f, 0.5f, 0.75f, 0.05f, 0.25f};
        rc = ping_pong(steps_, d_temp_, d_ref_, d_work_, [&](int, const float* src, float* dst) {
            return launch_hotspot_reference_step(s_.rows, s_.cols, src, d_power_, dst, hs_fold(k_), stream_);
        });
        if (rc) return rc;
        // Copies of (temperature, power, output, work) for sustained timing:
        // together at least 512 MiB (twice the last-level cache), at most 8.
        const size_t set_bytes = 16 * n_;
        const size_t n_sets = std::min<size_t>(8, std::max<size_t>(1, ((512ull << 20) + set_bytes - 1) / set_bytes));
        sets_.assign(1, {d_temp_, d_power_, d_out_, d_work_});
        for (size_t k = 1; k < n_sets; ++k) {
            std::array<float*, 4> b{};
            for (float*& p : b)
                if (hipMalloc(&p, n_ * 4) != hipSuccess) {
                    for (float* q : b)
                        if (q) hipFree(q);
                    return fail(CONV2D_ENOMEM, "hotspot tuner: device allocation");
                }
            sets_.push_back(b);
            rc = launch_fill_uniform(b[0], n_, 11, 0, stream_);
            if (!rc) rc = launch_fill_uniform(b[1], n_, 12, 0, stream_);
            if (rc) return rc;
        }
        CONV2D_HIP(hipStreamSynchronize(stream_));
        return CONV2D_OK;
    }

    void set_sustained(bool on) override { sustained_ = on; }

    int prepare(const std::vector<hotspot_config>& cfgs, std::vector<int>* status, double* seconds) override
    {
        const double t0 = now_s();
        status->assign(cfgs.size(), kOk);
        code_.assign(cfgs.size(), {});
        index_.clear();
        for (size_t i = 0; i < cfgs.size(); ++i) index_[hs_str(cfgs[i])] = i;
        int nthreads = o_.threads > 0 ? o_.threads : (int)std::thread::hardware_concurrency();
        nthreads = std::max(1, std::min(nthreads, 16));
        std::atomic<size_t> next{0};
        std::vector<std::thread> pool;
        for (int t = 0; t < nthreads; ++t)
            pool.emplace_back([&] {
                for (;;) {
                    const size_t i = next++;
                    if (i >= cfgs.size()) break;
                    if (hs_compile(cfgs[i], dev_.arch, &code_[i], nullptr) != CONV2D_OK) (*status)[i] = kCompile;
                }
            });
        for (auto& th : pool) th.join();
        *seconds = now_s() - t0;
        if (o_.verbose)
            std::fprintf(stderr, "[hotspot tune] compiled %zu configurations in %.1f s\n", cfgs.size(), *seconds);
        return CONV2D_OK;
    }

    int measure(const hotspot_config& c, int warmup, int reps, double best_so_far,
                RecordT<hotspot_config>* r) override
    {
        r->c = c;
        auto it = index_.find(hs_str(c));
        if (it == index_.end()) return fail(CONV2D_EINVAL, "hotspot config not prepared");
        Module m;
        if (load_module(code_[it->second], hs_kernel_name(c), &m) != CONV2D_OK) {
            r->status = kLaunch;
            return CONV2D_OK;
        }
        std::vector<char>().swap(code_[it->second]);
        int rc = run_checked(m, c, r);
        if (rc == CONV2D_OK && r->status == kOk) rc = time_it(m, c, warmup, reps, best_so_far, r);
        unload_module(&m);
        return rc;
    }

private:
    int run(const Module& m, const hotspot_config& c, size_t set = 0)
    {
        const auto& b = sets_[set];
        return hs_run(m, c, s_, b[0], b[1], b[2], b[3], steps_, k_, stream_);
    }

    int run_checked(const Module& m, const hotspot_config& c, RecordT<hotspot_config>* r)
    {
        int rc = launch_fill_value(d_out_, n_, __builtin_nanf(""), stream_);
        if (rc) return rc;
        if (run(m, c) != CONV2D_OK) {
            (void)hipGetLastError();
            r->status = kLaunch;
            return CONV2D_OK;
        }
        hipError_t e = hipStreamSynchronize(stream_);
        if (e != hipSuccess) return hip_fail(e, "hotspot tuner: kernel execution");
        CONV2D_HIP(hipMemsetAsync(d_count_, 0, sizeof(unsigned), stream_));
        rc = launch_count_mismatch(d_out_, d_ref_, n_, d_count_, stream_);
        if (rc) return rc;
        unsigned bad = 0;
        CONV2D_HIP(hipMemcpyAsync(&bad, d_count_, sizeof bad, hipMemcpyDeviceToHost, stream_));
        CONV2D_HIP(hipStreamSynchronize(stream_));
        r->status = bad ? kVerify : kOk;
        return CONV2D_OK;
    }

    int time_it(const Module& m, const hotspot_config& c, int warmup, int reps, double best_so_far,
                RecordT<hotspot_config>* r)
    {
        if (sustained_) {
            const size_t n = sets_.size();
            for (int k = 0; k < warmup + (int)n; ++k)
                if (run(m, c, (size_t)k % n)) return fail(CONV2D_ELAUNCH, "hotspot tuner: warm-up run failed");
            CONV2D_HIP(hipEventRecord(e0_, stream_));
            for (int k = 0; k < reps; ++k)
                if (run(m, c, (size_t)k % n)) return fail(CONV2D_ELAUNCH, "hotspot tuner: timed run failed");
            CONV2D_HIP(hipEventRecord(e1_, stream_));
            CONV2D_HIP(hipEventSynchronize(e1_));
            float ms = 0;
            CONV2D_HIP(hipEventElapsedTime(&ms, e0_, e1_));
            r->ms = r->ms_min = r->ms_p90 = ms / reps;
            r->reps = reps;
            return CONV2D_OK;
        }
        for (int k = 0; k < warmup; ++k)
            if (run(m, c)) return fail(CONV2D_ELAUNCH, "hotspot tuner: warm-up run failed");
        std::vector<double> t;
        for (int k = 0; k < reps; ++k) {
            if (d_flush_ && launch_flush(d_flush_, n_flush_, stream_)) return CONV2D_ELAUNCH;
            CONV2D_HIP(hipEventRecord(e0_, stream_));
            if (run(m, c)) return fail(CONV2D_ELAUNCH, "hotspot tuner: timed run failed");
            CONV2D_HIP(hipEventRecord(e1_, stream_));
            CONV2D_HIP(hipEventSynchronize(e1_));
            float ms = 0;
            CONV2D_HIP(hipEventElapsedTime(&ms, e0_, e1_));
            t.push_back(ms);
            if (best_so_far > 0 && k >= 2 && t[0] > 20.0 * best_so_far) break;
        }
        r->ms = median_of(t);
        r->ms_min = *std::min_element(t.begin(), t.end());
        r->ms_p90 = quantile_nearest(t, 0.9);
        r->reps = (int)t.size();
        return CONV2D_OK;
    }

    hotspot_shape s_;
    int steps_;
    hotspot_tune_opts o_;
    DeviceInfo dev_;
    hotspot_coeffs k_{};
    size_t n_ = 0, n_flush_ = 0;
    float *d_temp_ = nullptr, *d_power_ = nullptr, *d_out_ = nullptr, *d_work_ = nullptr, *d_ref_ = nullptr,
          *d_flush_ = nullptr;
    unsigned* d_count_ = nullptr;
    hipStream_t stream_ = nullptr;
    hipEvent_t e0_ = nullptr, e1_ = nullptr;
    std::vector<std::vector<char>> code_;
    std::map<std::string, size_t> index_;
    std::vector<std::array<float*, 4>> sets_;   // set 0: the buffers above
    bool sustained_ = false;
};

void load_hs_results(const std::string& path, const std::string& arch, const hotspot_shape& s, int steps,
                     std::map<std::string, RecordT<hotspot_config>>* out)
{
    std::ifstream f(path);
    if (!f) return;
    const std::string src = hex64(hs_source_hash());
    std::string line;
    while (std::getline(f, line)) {
        JsonObj o;
        if (!json_parse_line(line, &o) || o.str["arch"] != arch || o.str["src"] != src || !json_grid_is(o, s) ||
            (int)o.num["steps"] != steps)
            continue;
        RecordT<hotspot_config> r;
        if (!json_hs_config(o, &r.c)) continue;
        r.status = status_from(o.str["status"]);
        r.ms = o.num["ms"];
        r.ms_min = o.num["ms_min"];
        r.ms_p90 = o.num["ms_p90"];
        r.reps = (int)o.num["reps"];
        (*out)[hs_str(r.c)] = r;
    }
}

}  // namespace

const std::string& hotspot_source() { return hs_source(); }

hs_terms hs_fold(const hotspot_coeffs& k)
{
    const double cc = k.cc, gx = k.gx, gy = k.gy, gz = k.gz, ta = k.t_amb;
    return hs_terms{(float)(1.0 - cc * (2.0 * gx + 2.0 * gy + gz)), (float)(cc * gy), (float)(cc * gx), k.cc,
                    (float)(cc * gz * ta)};
}

}  // namespace conv2d

using namespace conv2d;

struct hotspot_plan_s {
    int device = -1;
    hotspot_shape shape{};
    hotspot_config cfg{};
    int tuned = 0;
    Module mod;
};

extern "C" void hotspot_default_config(hotspot_config* cfg)
{
    if (cfg) *cfg = hotspot_config{32, 8, 1, 1, 1, 1, 1};
}

extern "C" int hotspot_lds_bytes(const hotspot_config* cfg)
{
    if (!cfg) return fail(CONV2D_EINVAL, "cfg is NULL");
    // block_x <= 64: two buffers of the thread rows' top and bottom cell rows
    // (two zero rows beside them); wider blocks: two buffers of the region
    // plus a one-cell ring, odd pitch
    const long long b = cfg->block_x <= 64
                            ? 2ll * (2 * cfg->block_y + 4) * region_cols(*cfg) * 4
                            : 2ll * (region_rows(*cfg) + 2) * ((region_cols(*cfg) + 2) | 1) * 4;
    return b > INT_MAX ? INT_MAX : (int)b;
}

extern "C" int hotspot_config_check(hotspot_shape s, const hotspot_config* cfg, int lds_limit)
{
    clear_error();
    if (!cfg) return fail(CONV2D_EINVAL, "cfg is NULL");
    int rc = shape_ok(s);
    if (rc) return rc;
    const hotspot_config& c = *cfg;
    if (!on_axis(c.block_x, kBlockX) || !on_axis(c.block_y, kBlockY) || !on_axis(c.tile_x, kTile) ||
        !on_axis(c.tile_y, kTile) || !on_axis(c.temporal, kTemporal) || !on_axis(c.unroll_t, kUnrollT) ||
        !on_axis(c.sh_power, kShPower))
        return fail(CONV2D_EINVAL, "hotspot config " + hs_str(c) + ": a value is not on its axis");
    const int nt = c.block_x * c.block_y;
    if (nt < 64 || nt > 1024)
        return fail(CONV2D_EINVAL, "hotspot config " + hs_str(c) + ": needs 64..1024 threads");
    if (region_rows(c) <= 2 * c.temporal || region_cols(c) <= 2 * c.temporal)
        return fail(CONV2D_EINVAL, "hotspot config " + hs_str(c) + ": region not larger than twice the temporal factor");
    const int limit = lds_limit > 0 ? lds_limit : kLdsLimitGfx950;
    if (hotspot_lds_bytes(&c) > limit)
        return fail(CONV2D_EINVAL, "hotspot config " + hs_str(c) + ": LDS above the limit");
    if (hs_geometry(s, c).n_tiles < 1) return fail(CONV2D_EINVAL, "hotspot: too many tiles for one launch");
    return CONV2D_OK;
}

extern "C" int hotspot_space(hotspot_shape s, int lds_limit, hotspot_config* out, int cap)
{
    clear_error();
    int rc = shape_ok(s);
    if (rc) return rc;
    int n = 0;
    for (int bx : kBlockX)
        for (int by : kBlockY)
            for (int tx : kTile)
                for (int ty : kTile)
                    for (int tt : kTemporal)
                        for (int u : kUnrollT)
                            for (int p : kShPower) {
                                const hotspot_config c{bx, by, tx, ty, tt, u, p};
                                if (hotspot_config_check(s, &c, lds_limit) != CONV2D_OK) continue;
                                if (out && n < cap) out[n] = c;
                                ++n;
                            }
    clear_error();
    return n;
}

extern "C" int hotspot_compile(const hotspot_config* cfg, char* path_out, int path_cap)
{
    clear_error();
    if (!cfg) return fail(CONV2D_EINVAL, "cfg is NULL");
    int rc = hotspot_config_check(hotspot_shape{1, 1}, cfg, 0);
    if (rc) return rc;
    std::string path;
    rc = hs_compile(*cfg, env_str("CONV2D_ARCH", "gfx950"), nullptr, &path);
    if (rc) return rc;
    if (path_out && path_cap > 0) {
        std::strncpy(path_out, path.c_str(), (size_t)path_cap - 1);
        path_out[path_cap - 1] = '\0';
    }
    return CONV2D_OK;
}

extern "C" const char* hotspot_kernel_hash(void)
{
    static const std::string h = hex64(hs_source_hash());
    return h.c_str();
}

extern "C" int hotspot_plan(hotspot_plan_t* out, hotspot_shape s, const hotspot_config* cfg)
{
    clear_error();
    if (!out) return fail(CONV2D_EINVAL, "plan is NULL");
    *out = nullptr;
    int rc = shape_ok(s);
    if (rc) return rc;
    DeviceInfo dev;
    rc = current_device_info(&dev);
    if (rc) return rc;
    std::unique_ptr<hotspot_plan_s> p(new hotspot_plan_s);
    p->device = dev.device;
    p->shape = s;
    if (cfg) {
        p->cfg = *cfg;
    } else {
        std::string wp = env_str("HOTSPOT_WINNERS");
        if (wp.empty()) wp = hs_winners_default_path();
        if (hs_cache_lookup(wp, dev.arch, s, &p->cfg, nullptr) == CONV2D_OK &&
            hotspot_config_check(s, &p->cfg, dev.lds_limit) == CONV2D_OK)
            p->tuned = 1;
        else if (hs_cache_lookup_other(wp, dev.arch, s, dev.lds_limit, &p->cfg) == CONV2D_OK)
            p->tuned = 2;
        else
            hotspot_default_config(&p->cfg);
        clear_error();
    }
    rc = hotspot_config_check(s, &p->cfg, dev.lds_limit);
    if (rc) return rc;
    std::vector<char> code;
    rc = hs_compile(p->cfg, dev.arch, &code, nullptr);
    if (rc) return rc;
    rc = load_module(code, hs_kernel_name(p->cfg), &p->mod);
    if (rc) return rc;
    *out = p.release();
    return CONV2D_OK;
}

extern "C" int hotspot_plan_config(hotspot_plan_t plan, hotspot_config* cfg, int* tuned)
{
    clear_error();
    if (!plan) return fail(CONV2D_EINVAL, "plan is NULL");
    if (cfg) *cfg = plan->cfg;
    if (tuned) *tuned = plan->tuned;
    return CONV2D_OK;
}

extern "C" int hotspot_run(hotspot_plan_t plan, const float* d_temp, const float* d_power, float* d_out,
                           float* d_work, int steps, hotspot_coeffs k, void* stream)
{
    clear_error();
    if (!plan) return fail(CONV2D_EINVAL, "plan is NULL");
    if (steps < 0) return fail(CONV2D_EINVAL, "steps must be >= 0");
    int dev = -1;
    CONV2D_HIP(hipGetDevice(&dev));
    if (dev != plan->device) return fail(CONV2D_EINVAL, "plan was made for another device");
    const int launches = steps == 0 ? 0 : (steps + plan->cfg.temporal - 1) / plan->cfg.temporal;
    int rc = check_buffers(plan->shape, d_temp, d_power, d_out, d_work, launches);
    if (rc) return rc;
    return hs_run(plan->mod, plan->cfg, plan->shape, d_temp, d_power, d_out, d_work, steps, k,
                  static_cast<hipStream_t>(stream));
}

namespace conv2d {
// hotspot_run with a work grid the caller vouches for (work_cells floats of
// device memory that overlaps none of the caller's buffers): the library's
// fixed work array of hotspot_run_noalloc. Allocates nothing.
int hotspot_run_fixed_work(hotspot_plan_t plan, const float* d_temp, const float* d_power, float* d_out,
                           float* work, size_t work_cells, int steps, hotspot_coeffs k, void* stream)
{
    if (!plan) return fail(CONV2D_EINVAL, "plan is NULL");
    if (steps < 0) return fail(CONV2D_EINVAL, "steps must be >= 0");
    int dev = -1;
    CONV2D_HIP(hipGetDevice(&dev));
    if (dev != plan->device) return fail(CONV2D_EINVAL, "plan was made for another device");
    const int launches = steps == 0 ? 0 : (steps + plan->cfg.temporal - 1) / plan->cfg.temporal;
    const size_t cells = (size_t)plan->shape.rows * (size_t)plan->shape.cols;
    if (launches > 1 && cells > work_cells)
        return fail(CONV2D_EINVAL, "grid of " + std::to_string(cells) + " cells exceeds the fixed work array of " +
                                       std::to_string(work_cells));
    // The caller's buffers as for one launch; the work array is the library's own.
    int rc = check_buffers(plan->shape, d_temp, d_power, d_out, nullptr, std::min(launches, 1));
    if (rc) return rc;
    return hs_run(plan->mod, plan->cfg, plan->shape, d_temp, d_power, d_out, work, steps, k,
                  static_cast<hipStream_t>(stream));
}
}  // namespace conv2d

extern "C" void hotspot_destroy(hotspot_plan_t plan)
{
    if (!plan) return;
    unload_module(&plan->mod);
    delete plan;
}

extern "C" int hotspot_reference(hotspot_shape s, const float* d_temp, const float* d_power, float* d_out,
                                 float* d_work, int steps, hotspot_coeffs k, void* stream)
{
    clear_error();
    int rc = shape_ok(s);
    if (rc) return rc;
    if (steps < 0) return fail(CONV2D_EINVAL, "steps must be >= 0");
    rc = check_buffers(s, d_temp, d_power, d_out, d_work, steps);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (steps == 0) {
        CONV2D_HIP(hipMemcpyAsync(d_out, d_temp, 4ull * (size_t)s.rows * (size_t)s.cols, hipMemcpyDeviceToDevice, st));
        return CONV2D_OK;
    }
    const hs_terms t = hs_fold(k);
    return ping_pong(steps, d_temp, d_out, d_work, [&](int, const float* src, float* dst) {
        return launch_hotspot_reference_step(s.rows, s.cols, src, d_power, dst, t, st);
    });
}

extern "C" void hotspot_tune_defaults(hotspot_tune_opts* o)
{
    if (!o) return;
    *o = hotspot_tune_opts{};
    o->warmup = 2;
    o->reps = 20;
    o->retime_reps = 200;
    o->flush_mall = 1;
    o->tie_rel = 0.005;
}

extern "C" int hotspot_tune(hotspot_shape s, int steps, const hotspot_tune_opts* opts, hotspot_tune_result* res)
{
    clear_error();
    if (!res) return fail(CONV2D_EINVAL, "res is NULL");
    *res = hotspot_tune_result{};
    int rc = shape_ok(s);
    if (rc) return rc;
    if (steps < 1) return fail(CONV2D_EINVAL, "tuning needs steps >= 1");
    hotspot_tune_opts o;
    hotspot_tune_defaults(&o);
    if (opts) o = *opts;
    o.warmup = std::max(0, o.warmup);
    o.reps = std::max(1, o.reps);
    o.retime_reps = std::max(0, o.retime_reps);
    o.tie_rel = std::max(0.0, o.tie_rel);

    HotspotMeasurer meas(s, steps, o);
    rc = meas.init();
    if (rc) return rc;

    const int n_space = hotspot_space(s, -1, nullptr, 0);
    std::vector<hotspot_config> space(n_space);
    hotspot_space(s, -1, space.data(), n_space);
    res->n_space = n_space;
    hotspot_config dflt;
    hotspot_default_config(&dflt);
    std::vector<hotspot_config> legal;
    bool default_in = false;
    for (const auto& c : space) {
        if (hotspot_config_check(s, &c, meas.lds_limit()) != CONV2D_OK) { res->n_illegal++; continue; }
        legal.push_back(c);
        default_in = default_in || hs_equal(c, dflt);
    }
    clear_error();
    if (o.max_configs > 0 && (int)legal.size() > o.max_configs) legal.resize(o.max_configs);
    std::vector<hotspot_config> candidates = legal;
    if (!default_in) candidates.push_back(dflt);   // timed for tuned/default, not eligible

    std::map<std::string, RecordT<hotspot_config>> done;
    if (o.results_path && *o.results_path) load_hs_results(o.results_path, meas.arch(), s, steps, &done);
    std::vector<hotspot_config> todo;
    for (const auto& c : candidates)
        if (!done.count(hs_str(c))) todo.push_back(c);
    res->n_resumed = (int)(candidates.size() - todo.size());

    const double flops = hs_flops(s, steps);
    auto gflops = [&](double ms) { return ms > 0 ? flops / (ms * 1e-3) / 1e9 : 0.0; };
    auto sink = [&](const RecordT<hotspot_config>& r) {
        if (o.results_path && *o.results_path)
            append_line(o.results_path, record_line(meas.arch(), s, steps, r, r.status == kOk ? gflops(r.ms) : 0.0));
    };
    const double t0 = now_s();
    double best = 0;
    for (const auto& kv : done)
        if (kv.second.status == kOk && (best == 0 || kv.second.ms < best)) best = kv.second.ms;
    rc = measure_all(todo, &meas, o.warmup, o.reps, o.verbose != 0, hs_str, sink, &done, &best, &res->compile_s);
    if (rc) return rc;

    std::set<std::string> legal_keys;
    for (const auto& c : legal) legal_keys.insert(hs_str(c));
    std::vector<RecordT<hotspot_config>> eligible;
    for (const auto& c : candidates) {
        const auto& r = done[hs_str(c)];
        if (r.status == kCompile) res->n_compile_fail++;
        else if (r.status == kLaunch) res->n_launch_fail++;
        else if (r.status == kVerify) res->n_verify_fail++;
        else if (legal_keys.count(hs_str(c))) eligible.push_back(r);
    }
    res->n_timed = (int)eligible.size();
    RecordT<hotspot_config> win;
    std::vector<RecordT<hotspot_config>> top;
    rc = retime_and_pick(&eligible, &meas, o.warmup, o.retime_reps, 10, o.tie_rel, hs_less, &top, &win);
    if (rc) return rc;
    res->measure_s = now_s() - t0 - res->compile_s;
    res->best = win.c;
    res->best_ms = win.ms;
    for (int k = 0; k < 5 && k < (int)top.size(); ++k) {
        res->top[k] = top[k].c;
        res->top_ms[k] = top[k].ms;
    }
    std::vector<double> perf;
    for (const auto& r : eligible) perf.push_back(gflops(r.ms));
    const double med = median_of(perf);
    res->median_gflops = med;
    res->median_ms = flops / (med * 1e9) * 1e3;
    res->best_gflops = gflops(win.ms);
    res->impact = *std::max_element(perf.begin(), perf.end()) / med;
    {
        const auto wit = done.find(hs_str(win.c));
        if (wit != done.end() && wit->second.status == kOk) res->best_sweep_ms = wit->second.ms;
    }
    // The default's sweep rank, and its time in the winner's timing mode.
    const auto dit = done.find(hs_str(dflt));
    if (dit != done.end() && dit->second.status == kOk) {
        res->default_sweep_ms = dit->second.ms;
        int faster = 0;
        for (const auto& r : eligible)
            if (r.ms < res->default_sweep_ms && !hs_equal(r.c, dflt)) ++faster;
        res->default_rank = faster + 1;
        res->default_ms = res->default_sweep_ms;
        if (o.retime_reps > 0) {
            RecordT<hotspot_config> d;
            rc = retime_one(dflt, static_cast<MeasurerT<hotspot_config>*>(&meas), o.warmup, o.retime_reps, &d);
            if (rc) return rc;
            res->default_ms = d.status == kOk ? d.ms : 0;
        }
        res->default_gflops = res->default_ms > 0 ? gflops(res->default_ms) : 0;
    }
    if (o.winners_path && *o.winners_path) {
        const std::string wp = o.winners_path;
        const size_t slash = wp.find_last_of('/');
        if (slash != std::string::npos) make_dirs(wp.substr(0, slash));
        char b[384];
        std::snprintf(b, sizeof b, "{\"arch\":\"%s\",\"src\":\"%s\",\"shape\":[%d,%d],\"steps\":%d,\"config\":[%s],\"ms\":%.6f}",
                      json_escape(meas.arch()).c_str(), hex64(hs_source_hash()).c_str(), s.rows, s.cols, steps,
                      hs_str(win.c).c_str(), win.ms);
        if (!append_line(wp, b)) return fail(CONV2D_EINVAL, "cannot write hotspot winners cache " + wp);
    }
    return CONV2D_OK;
}
