// Serving: a trace of convolution requests (arrival time, shape, seeds) run
// with continuous batching, or one at a time through the plain path.
//
// Continuous batching. Arrived requests queue FIFO and are admitted while
// their device memory (input + filter + output) fits the HBM budget; an
// admitted request's image and filter are generated on the device (the stand
// in for an image that arrives in HBM). Whenever one of K streams is free, all
// admitted requests not yet launched (up to max_batch) go out as one batch:
// one fill launch for every image and filter of the batch, then one
// batched kernel per filter size and configuration present (each request
// takes its filter size's and size bucket's tuned configuration). Batches on different
// streams overlap on the device; completion is observed with events, and each
// request's latency runs from its arrival to the host seeing its batch done.
//
// Serial plain. The same trace, FIFO, one request at a time: fill, one
// conv2d_direct launch with the tuned configuration of its filter size, wait.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <numeric>
#include <tuple>
#include <thread>

#include "internal.h"

namespace conv2d {
namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// Best-fit bookkeeping over one device allocation (offsets only).
class Arena {
public:
    ~Arena()
    {
        if (base_) hipFree(base_);
    }
    int init(size_t bytes)
    {
        bytes = align_up(bytes);
        if (hipMalloc((void**)&base_, bytes) != hipSuccess) {
            base_ = nullptr;
            return fail(CONV2D_ENOMEM, "serve: cannot allocate the HBM budget arena");
        }
        free_[0] = bytes;
        return CONV2D_OK;
    }
    bool alloc(size_t n, size_t* off)
    {
        n = align_up(n);
        auto best = free_.end();
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n && (best == free_.end() || it->second < best->second)) best = it;
        if (best == free_.end()) return false;
        *off = best->first;
        const size_t len = best->second;
        free_.erase(best);
        if (len > n) free_[*off + n] = len - n;
        return true;
    }
    void release(size_t off, size_t n)
    {
        n = align_up(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    char* base() const { return base_; }

private:
    char* base_ = nullptr;
    std::map<size_t, size_t> free_;
};

struct Req {
    size_t off = 0, bytes = 0;
    float *in = nullptr, *f = nullptr, *out = nullptr;
    size_t n_in = 0, n_f = 0, n_out = 0;
    double t_launch = 0, t_done = 0;
    bool stalled = false;
    int kernel = -1;   // batched kernel of the request (index into the server's kernels)
};

struct FilterKernel {
    int fh = 0, fw = 0;
    conv2d_config cfg{};
    Module mod;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    std::vector<int> reqs;
    char* h_tab = nullptr;   // pinned: [fill descs | conv descs | owners]
    char* d_tab = nullptr;
    size_t cap = 0;
};

double percentile(std::vector<double> v, double p)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t rank = (size_t)std::ceil(p / 100.0 * (double)v.size());
    if (rank < 1) rank = 1;
    return v[std::min(rank, v.size()) - 1];
}

class Server {
public:
    Server(const conv2d_request* reqs, int n, const conv2d_serve_opts& o) : rq_(reqs), n_(n), o_(o) {}

    ~Server()
    {
        for (auto& s : slots_) {
            if (s.st) hipStreamSynchronize(s.st);
            if (s.ev) hipEventDestroy(s.ev);
            if (s.st) hipStreamDestroy(s.st);
            if (s.h_tab) hipHostFree(s.h_tab);
            if (s.d_tab) hipFree(s.d_tab);
        }
        for (auto& k : kernels_) unload_module(&k.mod);
        for (auto& kv : direct_) unload_module(&kv.second);
        // Kept outputs belong to the caller only once run() has handed them
        // over; after an error they are freed here (the streams are idle).
        if (!outputs_handed_)
            for (auto& r : req_)
                if (o_.keep_outputs && r.out) hipFree(r.out);
    }

    int init()
    {
        int rc = current_device_info(&dev_);
        if (rc) return rc;
        req_.assign(n_, Req{});
        size_t max_tiles_per_req = 1;
        for (int i = 0; i < n_; ++i) {
            const conv2d_shape& s = rq_[i].shape;
            rc = shape_check(s);
            if (rc) return fail(rc, "request " + std::to_string(i) + ": " + last_error_cstr());
            Req& r = req_[i];
            r.n_in = ((size_t)s.out_h + s.filt_h - 1) * ((size_t)s.out_w + s.filt_w - 1);
            r.n_f = (size_t)s.filt_h * s.filt_w;
            r.n_out = (size_t)s.out_h * s.out_w;
            if (r.n_in * 4 > (size_t)INT32_MAX) return fail(CONV2D_EINVAL, "request input above 2 GiB");
            r.bytes = align_up(r.n_in * 4) + align_up(r.n_f * 4) + (o_.keep_outputs ? 0 : align_up(r.n_out * 4));
            if (r.bytes > o_.hbm_budget)
                return fail(CONV2D_EINVAL, "request " + std::to_string(i) + " alone exceeds the HBM budget");
            // Kernels for every filter size and size bucket of the trace are
            // built up front (buckets that share a configuration share one).
            if (!o_.serial_plain) {
                const auto bkey = std::make_tuple(s.filt_h, s.filt_w, size_bucket(s.out_h, s.out_w));
                auto it = kernel_of_bucket_.find(bkey);
                if (it == kernel_of_bucket_.end()) {
                    const conv2d_config c = batch_config_for(dev_, s.filt_h, s.filt_w, std::get<2>(bkey), 0);
                    const auto ckey = std::make_pair(std::make_pair(s.filt_h, s.filt_w), config_str(c));
                    auto jt = kernel_of_cfg_.find(ckey);
                    if (jt == kernel_of_cfg_.end()) {
                        FilterKernel fk;
                        fk.fh = s.filt_h;
                        fk.fw = s.filt_w;
                        fk.cfg = c;
                        rc = batch_module(dev_, s.filt_h, s.filt_w, &fk.cfg, &fk.mod);
                        if (rc) return rc;
                        kernels_.push_back(fk);
                        jt = kernel_of_cfg_.emplace(ckey, (int)kernels_.size() - 1).first;
                    }
                    it = kernel_of_bucket_.emplace(bkey, jt->second).first;
                }
                req_[i].kernel = it->second;
                const conv2d_config& c = kernels_[(size_t)it->second].cfg;
                max_tiles_per_req = std::max(max_tiles_per_req, (size_t)geometry(s.out_h, s.out_w, c).n_tiles);
            }
        }
        // The serial baseline's modules for every (filter, alignment) class,
        // built before the clock starts so compilation is not charged to the
        // requests (the batched kernels were built above).
        if (o_.serial_plain) {
            for (int i = 0; i < n_; ++i) {
                conv2d_config c;
                const Module* m;
                rc = direct_module(rq_[i].shape, &c, &m);
                if (rc) return rc;
            }
        }
        rc = arena_.init(o_.hbm_budget);
        if (rc) return rc;
        const int n_slots = o_.serial_plain ? 1 : o_.streams;
        slots_.resize(n_slots);
        const size_t mb = (size_t)std::min(o_.max_batch, std::max(n_, 1));
        for (auto& s : slots_) {
            CONV2D_HIP(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
            CONV2D_HIP(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
            s.cap = 2 * mb * sizeof(FillDesc) + mb * sizeof(ConvDesc) + mb * max_tiles_per_req * sizeof(unsigned short) +
                    256;
            if (hipHostMalloc((void**)&s.h_tab, s.cap, hipHostMallocDefault) != hipSuccess ||
                hipMalloc((void**)&s.d_tab, s.cap) != hipSuccess)
                return fail(CONV2D_ENOMEM, "serve: descriptor tables");
        }
        return CONV2D_OK;
    }

    int run(conv2d_serve_report* rep, double* lat_ms, float** outs)
    {
        const auto t0 = std::chrono::steady_clock::now();
        auto now = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
        int rc = o_.serial_plain ? run_serial(now) : run_batched(now);
        if (rc) return rc;
        // Report.
        std::vector<double> lat(n_), queue(n_);
        double flops = 0, last = 0;
        for (int i = 0; i < n_; ++i) {
            lat[i] = 1e3 * (req_[i].t_done - rq_[i].arrival_s);
            queue[i] = 1e3 * (req_[i].t_launch - rq_[i].arrival_s);
            const conv2d_shape& s = rq_[i].shape;
            flops += 2.0 * s.out_h * (double)s.out_w * s.filt_h * s.filt_w;
            last = std::max(last, req_[i].t_done);
            if (lat_ms) lat_ms[i] = lat[i];
            if (outs) outs[i] = o_.keep_outputs ? req_[i].out : nullptr;
        }
        outputs_handed_ = true;
        *rep = conv2d_serve_report{};
        rep->n_requests = n_;
        rep->n_batches = n_batches_;
        rep->wall_s = n_ ? last - rq_[0].arrival_s : 0.0;
        rep->req_per_s = rep->wall_s > 0 ? n_ / rep->wall_s : 0.0;
        rep->gflops = rep->wall_s > 0 ? flops / rep->wall_s / 1e9 : 0.0;
        rep->offered_rate = (n_ > 1 && rq_[n_ - 1].arrival_s > rq_[0].arrival_s)
                                ? (n_ - 1) / (rq_[n_ - 1].arrival_s - rq_[0].arrival_s) : 0.0;
        rep->p50_ms = percentile(lat, 50);
        rep->p99_ms = percentile(lat, 99);
        rep->max_ms = percentile(lat, 100);
        rep->mean_ms = n_ ? std::accumulate(lat.begin(), lat.end(), 0.0) / n_ : 0.0;
        rep->queue_p50_ms = percentile(queue, 50);
        rep->queue_p99_ms = percentile(queue, 99);
        rep->mean_batch = n_batches_ ? (double)n_ / n_batches_ : 0.0;
        rep->stalled_requests = stalled_;
        rep->peak_bytes = peak_;
        rep->late_start_ms = 1e3 * late_start_;
        return CONV2D_OK;
    }

private:
    // ---------------------------------------------------------------- memory
    // 1: admitted; 0: wait for in-flight requests to release budget or arena
    // space; CONV2D_ENOMEM: it cannot be admitted by waiting (a kept output's
    // own allocation failed, or the arena is empty and still has no room).
    int admit(int i)
    {
        Req& r = req_[i];
        if (in_flight_ + r.bytes > o_.hbm_budget) return in_flight_ ? 0 : no_room(i);
        if (!arena_.alloc(r.bytes, &r.off)) return in_flight_ ? 0 : no_room(i);
        char* p = arena_.base() + r.off;
        r.in = reinterpret_cast<float*>(p);
        r.f = reinterpret_cast<float*>(p + align_up(r.n_in * 4));
        if (o_.keep_outputs) {
            // Kept outputs live outside the arena until the caller frees them,
            // so retiring requests cannot make room for this one.
            if (hipMalloc((void**)&r.out, std::max<size_t>(r.n_out * 4, 4)) != hipSuccess) {
                (void)hipGetLastError();
                r.out = nullptr;
                arena_.release(r.off, r.bytes);
                return fail(CONV2D_ENOMEM, "serve: output allocation of request " + std::to_string(i));
            }
        } else {
            r.out = reinterpret_cast<float*>(p + align_up(r.n_in * 4) + align_up(r.n_f * 4));
        }
        in_flight_ += r.bytes;
        peak_ = std::max(peak_, in_flight_);
        return 1;
    }

    int no_room(int i)
    {
        return fail(CONV2D_ENOMEM, "serve: request " + std::to_string(i) + " does not fit the empty arena");
    }

    void retire(int i, double t)
    {
        Req& r = req_[i];
        r.t_done = t;
        arena_.release(r.off, r.bytes);
        in_flight_ -= r.bytes;
        ++done_;
    }

    // ---------------------------------------------------------------- batched
    int launch_batch(Slot& s, const std::vector<int>& batch, double t)
    {
        // Table layout: fill descriptors, conv descriptors (grouped by filter
        // size), tile owners (grouped likewise).
        const size_t nb = batch.size();
        FillDesc* fill = reinterpret_cast<FillDesc*>(s.h_tab);
        ConvDesc* desc = reinterpret_cast<ConvDesc*>(s.h_tab + 2 * nb * sizeof(FillDesc));
        unsigned short* owner = reinterpret_cast<unsigned short*>(s.h_tab + 2 * nb * sizeof(FillDesc) +
                                                                  nb * sizeof(ConvDesc));
        unsigned long long max_n = 0;
        for (size_t k = 0; k < nb; ++k) {
            const Req& r = req_[batch[k]];
            fill[2 * k] = FillDesc{r.in, r.n_in, rq_[batch[k]].seed_in, 0};
            fill[2 * k + 1] = FillDesc{r.f, r.n_f, rq_[batch[k]].seed_f, 0};
            max_n = std::max<unsigned long long>(max_n, r.n_in);
        }
        struct G {
            const FilterKernel* fk;
            size_t d0, dn, o0;
            int tiles;
        };
        std::vector<G> groups;
        std::map<int, std::vector<int>> by_kernel;
        for (int i : batch) by_kernel[req_[i].kernel].push_back(i);
        size_t nd = 0, no = 0;
        for (auto& kv : by_kernel) {
            const FilterKernel& fk = kernels_.at((size_t)kv.first);
            G g{&fk, nd, kv.second.size(), no, 0};
            for (size_t k = 0; k < kv.second.size(); ++k) {
                const int i = kv.second[k];
                const conv2d_shape& sh = rq_[i].shape;
                const Req& r = req_[i];
                Geometry geo = geometry(sh.out_h, sh.out_w, fk.cfg);
                ConvDesc& d = desc[nd + k];
                d = ConvDesc{r.in, r.f, r.out, sh.out_h, sh.out_w, geo.tiles_x, g.tiles, (unsigned)(r.n_in * 4),
                             geo.n_tiles};
                std::fill(owner + no, owner + no + geo.n_tiles, (unsigned short)k);
                no += geo.n_tiles;
                g.tiles += geo.n_tiles;
            }
            nd += kv.second.size();
            groups.push_back(g);
        }
        const size_t bytes = 2 * nb * sizeof(FillDesc) + nb * sizeof(ConvDesc) + no * sizeof(unsigned short);
        if (bytes > s.cap) return fail(CONV2D_EINVAL, "serve: batch tables exceed their capacity");
        CONV2D_HIP(hipMemcpyAsync(s.d_tab, s.h_tab, bytes, hipMemcpyHostToDevice, s.st));
        const FillDesc* d_fill = reinterpret_cast<const FillDesc*>(s.d_tab);
        const ConvDesc* d_desc = reinterpret_cast<const ConvDesc*>(s.d_tab + 2 * nb * sizeof(FillDesc));
        const unsigned short* d_owner =
            reinterpret_cast<const unsigned short*>(s.d_tab + 2 * nb * sizeof(FillDesc) + nb * sizeof(ConvDesc));
        int rc = launch_fill_uniform_batch(d_fill, (int)(2 * nb), max_n, s.st);
        if (rc) return rc;
        for (const G& g : groups) {
            const int grid = std::max(8, g.tiles);   // one workgroup per tile, as the batched path
            rc = launch_batch_kernel(g.fk->mod, g.fk->cfg, grid, d_desc + g.d0, d_owner + g.o0, g.tiles, s.st);
            if (rc) return rc;
        }
        CONV2D_HIP(hipEventRecord(s.ev, s.st));
        s.busy = true;
        s.reqs = batch;
        for (int i : batch) req_[i].t_launch = t;
        ++n_batches_;
        return CONV2D_OK;
    }

    template <class Now>
    int run_batched(Now now)
    {
        std::deque<int> pending;
        std::vector<int> admitted;
        int next = 0;
        while (done_ < n_) {
            const double t = now();
            bool progress = false;
            while (next < n_ && rq_[next].arrival_s <= t) pending.push_back(next++);
            for (auto& s : slots_) {
                if (!s.busy) continue;
                hipError_t e = hipEventQuery(s.ev);
                if (e == hipErrorNotReady) continue;
                if (e != hipSuccess) return hip_fail(e, "serve: batch execution");
                const double td = now();
                for (int i : s.reqs) retire(i, td);
                s.busy = false;
                s.reqs.clear();
                progress = true;
            }
            while (!pending.empty()) {
                const int i = pending.front();
                const int a = admit(i);
                if (a < 0) return a;
                if (a == 0) {
                    if (!req_[i].stalled) { req_[i].stalled = true; ++stalled_; }
                    break;
                }
                pending.pop_front();
                admitted.push_back(i);
                progress = true;
            }
            if (!admitted.empty()) {
                for (auto& s : slots_) {
                    if (s.busy) continue;
                    const size_t take = std::min<size_t>(admitted.size(), (size_t)o_.max_batch);
                    std::vector<int> batch(admitted.begin(), admitted.begin() + take);
                    admitted.erase(admitted.begin(), admitted.begin() + take);
                    int rc = launch_batch(s, batch, now());
                    if (rc) return rc;
                    progress = true;
                    break;
                }
            }
            if (!progress) idle_wait(now, next, pending.empty() && admitted.empty());
        }
        return CONV2D_OK;
    }

    // Nothing to do: sleep towards the next arrival when the device is idle,
    // else yield briefly before polling again.
    template <class Now>
    void idle_wait(Now now, int next, bool nothing_queued)
    {
        bool any_busy = false;
        for (auto& s : slots_) any_busy = any_busy || s.busy;
        if (!any_busy && nothing_queued && next < n_) {
            const double wait = rq_[next].arrival_s - now();
            if (wait > 200e-6) std::this_thread::sleep_for(std::chrono::duration<double>(wait - 100e-6));
            return;
        }
        std::this_thread::yield();
    }

    // ---------------------------------------------------------------- serial plain
    int direct_module(const conv2d_shape& s, conv2d_config* cfg, const Module** m)
    {
        const auto key = std::make_tuple(s.filt_h, s.filt_w, kVec, kVec);
        auto fit = direct_cfg_.find({s.filt_h, s.filt_w});
        if (fit == direct_cfg_.end()) {
            std::string wp = env_str("CONV2D_WINNERS");
            if (wp.empty()) wp = winners_default_path();
            conv2d_config c;
            const conv2d_shape tuned{4096, 4096, s.filt_h, s.filt_w};
            if (cache_lookup_filter(wp, dev_.arch, s.filt_h, s.filt_w, tuned, &c) != CONV2D_OK ||
                conv2d_config_check(tuned, &c, dev_.lds_limit) != CONV2D_OK)
                conv2d_default_config(&c);
            clear_error();
            fit = direct_cfg_.emplace(std::make_pair(s.filt_h, s.filt_w), c).first;
        }
        *cfg = fit->second;
        auto it = direct_.find(key);
        if (it == direct_.end()) {
            conv2d_config built = *cfg;  // only the unroll may change, not the geometry
            Module mod;
            int rc = build_module(s, &built, kVec, kVec, dev_.arch, false, true, &mod);
            if (rc) return rc;
            it = direct_.emplace(key, mod).first;
        }
        *m = &it->second;
        return CONV2D_OK;
    }

    template <class Now>
    int run_serial(Now now)
    {
        Slot& s = slots_[0];
        FillDesc* fill = reinterpret_cast<FillDesc*>(s.h_tab);
        for (int i = 0; i < n_; ++i) {
            const double wait = rq_[i].arrival_s - now();
            if (wait > 200e-6) std::this_thread::sleep_for(std::chrono::duration<double>(wait - 100e-6));
            while (now() < rq_[i].arrival_s) std::this_thread::yield();
            const int a = admit(i);
            if (a < 0) return a;
            if (a == 0) return fail(CONV2D_ENOMEM, "serve: arena fragmentation in the serial run");
            Req& r = req_[i];
            r.t_launch = now();
            fill[0] = FillDesc{r.in, r.n_in, rq_[i].seed_in, 0};
            fill[1] = FillDesc{r.f, r.n_f, rq_[i].seed_f, 0};
            CONV2D_HIP(hipMemcpyAsync(s.d_tab, s.h_tab, 2 * sizeof(FillDesc), hipMemcpyHostToDevice, s.st));
            int rc = launch_fill_uniform_batch(reinterpret_cast<const FillDesc*>(s.d_tab), 2, r.n_in, s.st);
            if (rc) return rc;
            conv2d_config c;
            const Module* m;
            rc = direct_module(rq_[i].shape, &c, &m);
            if (rc) return rc;
            if (c.filter_in_const)
                CONV2D_HIP(hipMemcpyAsync(m->const_filter, r.f, r.n_f * 4, hipMemcpyDeviceToDevice, s.st));
            rc = launch_direct(*m, rq_[i].shape, c, r.in, r.f, r.out, s.st);
            if (rc) return rc;
            CONV2D_HIP(hipEventRecord(s.ev, s.st));
            CONV2D_HIP(hipEventSynchronize(s.ev));
            retire(i, now());
            ++n_batches_;
            late_start_ = std::max(late_start_, r.t_launch - rq_[i].arrival_s);
        }
        return CONV2D_OK;
    }

    const conv2d_request* rq_;
    int n_;
    conv2d_serve_opts o_;
    DeviceInfo dev_;
    std::vector<Req> req_;
    std::vector<FilterKernel> kernels_;
    std::map<std::tuple<int, int, int>, int> kernel_of_bucket_;
    std::map<std::pair<std::pair<int, int>, std::string>, int> kernel_of_cfg_;
    std::map<std::pair<int, int>, conv2d_config> direct_cfg_;
    std::map<std::tuple<int, int, int, int>, Module> direct_;
    Arena arena_;
    std::vector<Slot> slots_;
    size_t in_flight_ = 0, peak_ = 0;
    int done_ = 0, n_batches_ = 0, stalled_ = 0;
    double late_start_ = 0;
    bool outputs_handed_ = false;
};

}  // namespace
}  // namespace conv2d

using namespace conv2d;

extern "C" void conv2d_serve_defaults(conv2d_serve_opts* o)
{
    if (!o) return;
    *o = conv2d_serve_opts{};
    o->hbm_budget = 8ull << 30;
    o->streams = 4;
    o->max_batch = 64;
    o->serial_plain = 0;
    o->keep_outputs = 0;
}

extern "C" int conv2d_serve(const conv2d_request* reqs, int n, const conv2d_serve_opts* opts,
                            conv2d_serve_report* rep, double* latency_ms, float** outputs)
{
    clear_error();
    if (!reqs || n < 1 || !rep) return fail(CONV2D_EINVAL, "serve: need n >= 1 requests and a report");
    conv2d_serve_opts o;
    conv2d_serve_defaults(&o);
    if (opts) o = *opts;
    if (o.streams < 1 || o.streams > 16) return fail(CONV2D_EINVAL, "serve: streams must be in 1..16");
    if (o.max_batch < 1 || o.max_batch > 32767) return fail(CONV2D_EINVAL, "serve: max_batch must be in 1..32767");
    if (o.hbm_budget < (1ull << 20)) return fail(CONV2D_EINVAL, "serve: HBM budget below 1 MiB");
    if (o.keep_outputs && !outputs) return fail(CONV2D_EINVAL, "serve: keep_outputs needs an outputs array");
    for (int i = 0; i < n; ++i) {
        const double t = reqs[i].arrival_s;
        if (!std::isfinite(t) || t < 0.0)
            return fail(CONV2D_EINVAL, "serve: request " + std::to_string(i) + " has no finite arrival time >= 0");
        if (i > 0 && t < reqs[i - 1].arrival_s)
            return fail(CONV2D_EINVAL, "serve: arrival times must be non-decreasing");
    }
    auto s = std::make_unique<Server>(reqs, n, o);
    int rc = s->init();
    if (!rc) rc = s->run(rep, latency_ms, outputs);
    return rc;
}

extern "C" void conv2d_serve_free(float** outputs, int n)
{
    if (!outputs) return;
    for (int i = 0; i < n; ++i)
        if (outputs[i]) {
            hipFree(outputs[i]);
            outputs[i] = nullptr;
        }
}
