// Batched path: many convolutions of uneven sizes in one hipGraph launch.
//
// Problems are grouped by filter size (compile-time in the kernel). Each
// group gets the tuned configuration of its filter size and one
// kernel that walks the group's tile list; the problems are described in
// device memory (pointers, sizes, first tile), so the graph is captured once
// at plan time, with the groups as parallel branches, and a run is one
// hipGraphLaunch (after a small descriptor upload when the caller's pointers
// changed since the last run).
#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>

#include "internal.h"
#include "search.h"

namespace conv2d {
namespace {

struct Group {
    int fh = 0, fw = 0;
    conv2d_config cfg{};
    Module mod;
    std::vector<int> problems;   // indices into the batch's shapes
    int total_tiles = 0;
    int grid = 0;
    int threads = 0;
    size_t desc_begin = 0;       // first descriptor of the group
    size_t owner_begin = 0;      // first owner entry of the group
    // kernel arguments, kept alive for graph capture and direct launches
    const void* a_desc = nullptr;
    const void* a_owner = nullptr;
    int a_total = 0;
};

}  // namespace
}  // namespace conv2d

using namespace conv2d;

struct conv2d_batch_s {
    int device = -1;
    DeviceInfo dev;
    int flags = 0;
    std::vector<conv2d_shape> shapes;
    std::vector<Group> groups;
    std::vector<int> desc_slot;          // problem -> descriptor index
    ConvDesc* h_desc = nullptr;          // pinned staging
    ConvDesc* d_desc = nullptr;
    unsigned short* d_owner = nullptr;
    std::vector<const void*> uploaded;   // pointers of the descriptors on the device
    hipEvent_t copied = nullptr;
    bool copy_pending = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::mutex mu;
};

static void batch_free(conv2d_batch_s* b)
{
    if (!b) return;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->copied) {
        hipEventSynchronize(b->copied);
        hipEventDestroy(b->copied);
    }
    for (auto& g : b->groups) unload_module(&g.mod);
    if (b->h_desc) hipHostFree(b->h_desc);
    if (b->d_desc) hipFree(b->d_desc);
    if (b->d_owner) hipFree(b->d_owner);
    delete b;
}

static int launch_group(const Group& g, hipStream_t st)
{
    return launch_batch_kernel(g.mod, g.cfg, g.grid, g.a_desc, g.a_owner, g.a_total, st);
}

// Captures every group's kernel as a parallel branch of one graph.
static int capture(conv2d_batch_s* b)
{
    std::vector<hipStream_t> streams(b->groups.size() + 1, nullptr);
    std::vector<hipEvent_t> events(b->groups.size() + 1, nullptr);
    int rc = CONV2D_OK;
    auto cleanup = [&] {
        for (auto s : streams)
            if (s) hipStreamDestroy(s);
        for (auto e : events)
            if (e) hipEventDestroy(e);
    };
    for (size_t k = 0; k < streams.size(); ++k) {
        if (hipStreamCreateWithFlags(&streams[k], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&events[k], hipEventDisableTiming) != hipSuccess) {
            cleanup();
            return fail(CONV2D_EHIP, "batch: cannot create capture streams");
        }
    }
    hipStream_t root = streams[0];
    hipError_t e = hipStreamBeginCapture(root, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { cleanup(); return hip_fail(e, "hipStreamBeginCapture"); }
    e = hipEventRecord(events[0], root);
    if (e != hipSuccess) rc = hip_fail(e, "hipEventRecord (capture fork)");
    for (size_t g = 0; g < b->groups.size() && rc == CONV2D_OK; ++g) {
        hipStream_t st = streams[g + 1];
        if ((e = hipStreamWaitEvent(st, events[0], 0)) != hipSuccess) {
            rc = hip_fail(e, "hipStreamWaitEvent (capture fork)");
            break;
        }
        rc = launch_group(b->groups[g], st);
        // The branch is joined back to the root stream even after a failed
        // launch, so that the capture can end.
        if ((e = hipEventRecord(events[g + 1], st)) != hipSuccess ||
            (e = hipStreamWaitEvent(root, events[g + 1], 0)) != hipSuccess) {
            if (rc == CONV2D_OK) rc = hip_fail(e, "capture join");
            break;
        }
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(root, &graph);
    if (rc == CONV2D_OK && e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
    if (rc == CONV2D_OK) {
        e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
    }
    if (graph) {
        if (rc == CONV2D_OK) b->graph = graph;
        else hipGraphDestroy(graph);
    }
    cleanup();
    return rc;
}

namespace conv2d {

// Winners-cache shape of the batched path's own tuning of a filter size:
// (0, 0, fh, fw) for problems of any size, (0, b, fh, fw) for size bucket b.
static conv2d_shape batch_key(int fh, int fw, int bucket) { return conv2d_shape{0, bucket, fh, fw}; }

static std::string winners_path_or_default(const char* given)
{
    if (given && *given) return given;
    std::string wp = env_str("CONV2D_WINNERS");
    return wp.empty() ? winners_default_path() : wp;
}

int size_bucket(int out_h, int out_w)
{
    const int side = std::max(out_h, out_w);
    int b = 1;
    for (int bound = 384; b < CONV2D_SIZE_BUCKETS && side > bound; bound *= 2) ++b;
    return b;
}

// The configuration the batched path uses for a filter size: with a size
// bucket (> 0), the bucket's entry, else the filter's whole-batch entry;
// without (bucket 0), the whole-batch entry, else the entry of the bucket
// `fallback_bucket`; then the 4096x4096 winner, else the default. The filter
// is read through its pointer.
static conv2d_config lookup_batch_config(const DeviceInfo& dev, const std::string& wp, int fh, int fw, int bucket,
                                         int fallback_bucket = 0)
{
    const conv2d_shape tuned_shape{4096, 4096, fh, fw};
    conv2d_config cfg{};
    auto entry = [&](int b) { return cache_lookup(wp, dev.arch, batch_key(fh, fw, b), &cfg, nullptr) == CONV2D_OK; };
    bool found = bucket > 0 ? entry(bucket) || entry(0) : entry(0) || (fallback_bucket > 0 && entry(fallback_bucket));
    if (!found) found = cache_lookup_filter(wp, dev.arch, fh, fw, tuned_shape, &cfg) == CONV2D_OK;
    if (!found) conv2d_default_config(&cfg);
    clear_error();
    cfg.filter_in_const = 0;  // each problem has its own filter
    if (conv2d_config_check(tuned_shape, &cfg, dev.lds_limit) != CONV2D_OK) {
        conv2d_default_config(&cfg);
        cfg.filter_in_const = 0;
        clear_error();
    }
    return cfg;
}

conv2d_config batch_config_for(const DeviceInfo& dev, int fh, int fw, int bucket, int fallback_bucket)
{
    return lookup_batch_config(dev, winners_path_or_default(nullptr), fh, fw, bucket, fallback_bucket);
}

// The batched kernel's problems have rows of every alignment; it takes the
// 4-wide loads and stores of every build.
static constexpr int kBatchVin = kVec, kBatchVout = kVec;

int batch_module(const DeviceInfo& dev, int fh, int fw, conv2d_config* cfg, Module* m)
{
    // With a fully unrolled row loop that can spill, the rolled loop is used.
    return build_module(conv2d_shape{4096, 4096, fh, fw}, cfg, kBatchVin, kBatchVout, dev.arch, true, true, m);
}

int launch_batch_kernel(const Module& m, const conv2d_config& cfg, int grid, const void* d_desc,
                        const void* d_owner, int total_tiles, hipStream_t st)
{
    const void* d = d_desc;
    const void* o = d_owner;
    int total = total_tiles;
    void* args[] = {&d, &o, &total};
    hipError_t e = hipModuleLaunchKernel(m.fn, (unsigned)grid, 1, 1, (unsigned)(cfg.block_x * cfg.block_y), 1, 1, 0,
                                         st, args, nullptr);
    if (e != hipSuccess) return fail(CONV2D_ELAUNCH, std::string("batch launch: ") + hipGetErrorString(e));
    return CONV2D_OK;
}

}  // namespace conv2d

extern "C" int conv2d_batch_plan(conv2d_batch_t* out, int n, const conv2d_shape* shapes, int flags)
{
    clear_error();
    if (!out) return fail(CONV2D_EINVAL, "batch is NULL");
    *out = nullptr;
    if (n < 1 || !shapes) return fail(CONV2D_EINVAL, "a batch needs n >= 1 shapes");
    if (n > 65535) return fail(CONV2D_EINVAL, "a batch holds at most 65535 problems");
    for (int i = 0; i < n; ++i) {
        int rc = shape_check(shapes[i]);
        if (rc) return fail(rc, "problem " + std::to_string(i) + ": " + last_error_cstr());
        const long long bytes = 4ll * (shapes[i].out_h + shapes[i].filt_h - 1) * (shapes[i].out_w + shapes[i].filt_w - 1);
        if (bytes > INT_MAX) return fail(CONV2D_EINVAL, "problem " + std::to_string(i) + ": input above 2 GiB");
    }
    std::unique_ptr<conv2d_batch_s, void (*)(conv2d_batch_s*)> b(new conv2d_batch_s, batch_free);
    int rc = current_device_info(&b->dev);
    if (rc) return rc;
    b->device = b->dev.device;
    b->flags = flags;
    b->shapes.assign(shapes, shapes + n);

    // Group by filter size and configuration, heaviest filters first. By
    // default a filter size takes its whole-batch entry (one kernel for all
    // its problems: a large mixed batch runs best so); CONV2D_BATCH_BY_SIZE
    // gives each problem its size bucket's entry (the buckets of a filter that
    // share a configuration share a kernel).
    using Key = std::pair<std::pair<int, int>, std::string>;
    std::map<std::tuple<int, int, int>, conv2d_config> chosen;
    std::map<Key, std::vector<int>> by_kernel;
    std::map<Key, conv2d_config> kernel_cfg;
    for (int i = 0; i < n; ++i) {
        const auto bk = std::make_tuple(shapes[i].filt_h, shapes[i].filt_w, size_bucket(shapes[i].out_h, shapes[i].out_w));
        auto it = chosen.find(bk);
        if (it == chosen.end()) {
            const int bucket = std::get<2>(bk);
            const conv2d_config c = (flags & CONV2D_BATCH_BY_SIZE)
                                        ? batch_config_for(b->dev, shapes[i].filt_h, shapes[i].filt_w, bucket, 0)
                                        : batch_config_for(b->dev, shapes[i].filt_h, shapes[i].filt_w, 0, bucket);
            it = chosen.emplace(bk, c).first;
        }
        const Key key{{shapes[i].filt_h, shapes[i].filt_w}, config_str(it->second)};
        by_kernel[key].push_back(i);
        kernel_cfg[key] = it->second;
    }
    std::vector<Key> keys;
    for (auto& kv : by_kernel) keys.push_back(kv.first);
    std::stable_sort(keys.begin(), keys.end(), [](const Key& a, const Key& c) {
        return a.first.first * a.first.second > c.first.first * c.first.second;
    });

    std::vector<unsigned short> owner;
    std::vector<ConvDesc> proto;
    b->desc_slot.assign(n, -1);
    for (const auto& key : keys) {
        Group g;
        g.fh = key.first.first;
        g.fw = key.first.second;
        g.problems = by_kernel[key];
        g.cfg = kernel_cfg[key];
        rc = batch_module(b->dev, g.fh, g.fw, &g.cfg, &g.mod);
        if (rc) return rc;
        g.threads = g.cfg.block_x * g.cfg.block_y;
        g.desc_begin = proto.size();
        g.owner_begin = owner.size();
        for (size_t k = 0; k < g.problems.size(); ++k) {
            const conv2d_shape& s = shapes[g.problems[k]];
            Geometry geo = geometry(s.out_h, s.out_w, g.cfg);
            ConvDesc d{};
            d.H = s.out_h;
            d.W = s.out_w;
            d.tiles_x = geo.tiles_x;
            d.tile_begin = g.total_tiles;
            d.in_bytes = (unsigned)(4ull * (s.out_h + s.filt_h - 1) * (s.out_w + s.filt_w - 1));
            d.n_tiles = geo.n_tiles;
            if ((long long)g.total_tiles + geo.n_tiles > INT_MAX)
                return fail(CONV2D_EINVAL, "batch: too many tiles in one filter group");
            g.total_tiles += geo.n_tiles;
            owner.insert(owner.end(), (size_t)geo.n_tiles, (unsigned short)k);
            b->desc_slot[g.problems[k]] = (int)proto.size();
            proto.push_back(d);
        }
        // One workgroup per tile: the hardware dispatcher hands out tiles as
        // slots free up, which balances the concurrent groups better than a
        // static share per resident workgroup (measured 5 % faster on the
        // 64-problem workload).
        g.grid = std::max(8, g.total_tiles);
        b->groups.push_back(std::move(g));
    }

    // Device tables: descriptors (pointers filled at run time) and tile owners.
    if (hipHostMalloc((void**)&b->h_desc, sizeof(ConvDesc) * n, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&b->d_desc, sizeof(ConvDesc) * n) != hipSuccess ||
        hipMalloc((void**)&b->d_owner, sizeof(unsigned short) * owner.size()) != hipSuccess)
        return fail(CONV2D_ENOMEM, "batch: allocation of the descriptor tables failed");
    std::memcpy(b->h_desc, proto.data(), sizeof(ConvDesc) * n);
    CONV2D_HIP(hipMemcpy(b->d_owner, owner.data(), sizeof(unsigned short) * owner.size(), hipMemcpyHostToDevice));
    CONV2D_HIP(hipEventCreateWithFlags(&b->copied, hipEventDisableTiming));
    for (auto& g : b->groups) {
        g.a_desc = b->d_desc + g.desc_begin;
        g.a_owner = b->d_owner + g.owner_begin;
        g.a_total = g.total_tiles;
    }
    if (!(flags & CONV2D_BATCH_NO_GRAPH)) {
        rc = capture(b.get());
        if (rc) return rc;
    }
    *out = b.release();
    return CONV2D_OK;
}

extern "C" int conv2d_batch_run(conv2d_batch_t b, const float* const* d_in, const float* const* d_f,
                                float* const* d_out, void* stream)
{
    clear_error();
    if (!b || !d_in || !d_f || !d_out) return fail(CONV2D_EINVAL, "batch and pointer arrays must be non-NULL");
    int dev = -1;
    CONV2D_HIP(hipGetDevice(&dev));
    if (dev != b->device) return fail(CONV2D_EINVAL, "batch was planned for another device");
    const int n = (int)b->shapes.size();
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(b->mu);

    std::vector<const void*> ptrs(3 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        ptrs[3 * i] = d_in[i];
        ptrs[3 * i + 1] = d_f[i];
        ptrs[3 * i + 2] = d_out[i];
    }
    if (ptrs != b->uploaded) {
        if (!(b->flags & CONV2D_BATCH_NO_PTR_CHECK)) {
            for (int i = 0; i < n; ++i) {
                const conv2d_shape& s = b->shapes[i];
                const size_t in_b = 4ull * ((size_t)s.out_h + s.filt_h - 1) * ((size_t)s.out_w + s.filt_w - 1);
                const size_t f_b = 4ull * s.filt_h * s.filt_w, o_b = 4ull * s.out_h * s.out_w;
                int rc = check_device_range(d_in[i], in_b, "d_in");
                if (!rc) rc = check_device_range(d_f[i], f_b, "d_filter");
                if (!rc) rc = check_device_range(d_out[i], o_b, "d_out");
                if (rc) return fail(rc, "problem " + std::to_string(i) + ": " + last_error_cstr());
                const uintptr_t o = (uintptr_t)d_out[i], a = (uintptr_t)d_in[i], f = (uintptr_t)d_f[i];
                if ((o < a + in_b && a < o + o_b) || (o < f + f_b && f < o + o_b))
                    return fail(CONV2D_EINVAL, "problem " + std::to_string(i) + ": d_out overlaps its inputs");
            }
        }
        // The staging buffer may still feed the previous upload.
        if (b->copy_pending) CONV2D_HIP(hipEventSynchronize(b->copied));
        for (int i = 0; i < n; ++i) {
            ConvDesc& d = b->h_desc[b->desc_slot[i]];
            d.in = d_in[i];
            d.filt = d_f[i];
            d.out = d_out[i];
        }
        CONV2D_HIP(hipMemcpyAsync(b->d_desc, b->h_desc, sizeof(ConvDesc) * n, hipMemcpyHostToDevice, st));
        CONV2D_HIP(hipEventRecord(b->copied, st));
        b->copy_pending = true;
        b->uploaded = ptrs;
    }
    if (b->exec) {
        hipError_t e = hipGraphLaunch(b->exec, st);
        if (e != hipSuccess) return fail(CONV2D_ELAUNCH, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        return CONV2D_OK;
    }
    for (const auto& g : b->groups) {
        int rc = launch_group(g, st);
        if (rc) return rc;
    }
    return CONV2D_OK;
}

extern "C" int conv2d_batch_info(conv2d_batch_t b, int* n_groups, int* total_tiles, int* filt, conv2d_config* cfgs,
                                 int* grids, int cap)
{
    clear_error();
    if (!b) return fail(CONV2D_EINVAL, "batch is NULL");
    int tiles = 0;
    for (size_t g = 0; g < b->groups.size(); ++g) {
        tiles += b->groups[g].total_tiles;
        if ((int)g < cap) {
            if (filt) { filt[2 * g] = b->groups[g].fh; filt[2 * g + 1] = b->groups[g].fw; }
            if (cfgs) cfgs[g] = b->groups[g].cfg;
            if (grids) grids[g] = b->groups[g].grid;
        }
    }
    if (n_groups) *n_groups = (int)b->groups.size();
    if (total_tiles) *total_tiles = tiles;
    return CONV2D_OK;
}

extern "C" void conv2d_batch_destroy(conv2d_batch_t b) { batch_free(b); }

extern "C" int conv2d_compile_batch(conv2d_shape s, const conv2d_config* cfg, char* path_out, int path_cap)
{
    clear_error();
    if (!cfg) return fail(CONV2D_EINVAL, "cfg is NULL");
    conv2d_config c = *cfg;
    c.filter_in_const = 0;
    int rc = conv2d_config_check(s, &c, 0);
    if (rc) return rc;
    std::string path;
    rc = compile_direct(s, c, kBatchVin, kBatchVout, env_str("CONV2D_ARCH", "gfx950"), nullptr, &path, true);
    if (rc) return rc;
    if (path_out && path_cap > 0) {
        std::strncpy(path_out, path.c_str(), (size_t)path_cap - 1);
        path_out[path_cap - 1] = '\0';
    }
    return CONV2D_OK;
}

// ---------------------------------------------------------------- batch tuning

namespace conv2d {
namespace {

// Candidates from the 4096x4096 sweep of a filter size (any kernel source;
// filter moved to its pointer; legal; no repeats): its `k` fastest verified
// points, then the fastest point of every workgroup tile area (block_x *
// tile_x * block_y * tile_y) not yet present, which gives small images
// configurations with more, smaller tiles.
std::vector<conv2d_config> sweep_candidates(const DeviceInfo& dev, const std::string& dir, int fh, int fw, int k)
{
    char name[128];
    std::snprintf(name, sizeof name, "/results_%s_4096x4096_%dx%d.jsonl", dev.arch.c_str(), fh, fw);
    std::ifstream f(dir + name);
    std::vector<std::pair<double, conv2d_config>> all;
    std::string line;
    while (std::getline(f, line)) {
        JsonObj o;
        if (!json_parse_line(line, &o) || o.str["arch"] != dev.arch || o.str["status"] != "ok") continue;
        auto sh = o.arr.find("shape"), cf = o.arr.find("config");
        if (sh == o.arr.end() || cf == o.arr.end() || sh->second.size() != 4 || cf->second.size() != 7) continue;
        if ((int)sh->second[0] != 4096 || (int)sh->second[1] != 4096 || (int)sh->second[2] != fh ||
            (int)sh->second[3] != fw)
            continue;
        const auto& v = cf->second;
        all.push_back({o.num["ms"], conv2d_config{(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], 0, (int)v[6]}});
    }
    std::stable_sort(all.begin(), all.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    std::vector<conv2d_config> out;
    const conv2d_shape s{4096, 4096, fh, fw};
    auto add = [&](const conv2d_config& c) {
        for (const auto& e : out)
            if (config_equal(e, c)) return false;
        if (conv2d_config_check(s, &c, dev.lds_limit) != CONV2D_OK) return false;
        out.push_back(c);
        return true;
    };
    for (const auto& e : all) {
        if ((int)out.size() >= k) break;
        add(e.second);
    }
    std::map<long long, bool> areas;
    for (const auto& c : out) areas[(long long)c.block_x * c.tile_x * c.block_y * c.tile_y] = true;
    for (const auto& e : all) {
        const conv2d_config& c = e.second;
        const long long area = (long long)c.block_x * c.tile_x * c.block_y * c.tile_y;
        if (!areas.count(area) && add(c)) areas[area] = true;
    }
    clear_error();
    return out;
}

// One group's problems of a batch on the device: seeded inputs and
// filters, reference outputs, outputs, and the descriptor and owner tables
// of the batched kernel for a configuration.
struct GroupBench {
    std::vector<conv2d_shape> shapes;
    std::vector<float*> in, f, out, ref;
    ConvDesc* d_desc = nullptr;
    unsigned short* d_owner = nullptr;
    unsigned* d_count = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int tiles = 0;

    ~GroupBench()
    {
        if (st) hipStreamSynchronize(st);
        for (auto* v : {&in, &f, &out, &ref})
            for (float* p : *v)
                if (p) hipFree(p);
        if (d_desc) hipFree(d_desc);
        if (d_owner) hipFree(d_owner);
        if (d_count) hipFree(d_count);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        if (st) hipStreamDestroy(st);
    }

    int init()
    {
        CONV2D_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        CONV2D_HIP(hipEventCreate(&e0));
        CONV2D_HIP(hipEventCreate(&e1));
        if (hipMalloc(&d_desc, sizeof(ConvDesc) * shapes.size()) != hipSuccess ||
            hipMalloc(&d_count, sizeof(unsigned)) != hipSuccess)
            return fail(CONV2D_ENOMEM, "batch tune: device allocation");
        for (size_t k = 0; k < shapes.size(); ++k) {
            const conv2d_shape& s = shapes[k];
            const size_t n_in = (size_t)(s.out_h + s.filt_h - 1) * (s.out_w + s.filt_w - 1);
            const size_t n_out = (size_t)s.out_h * s.out_w;
            float *a = nullptr, *b = nullptr, *c = nullptr, *d = nullptr;
            if (hipMalloc(&a, n_in * 4) != hipSuccess || hipMalloc(&b, 4ull * s.filt_h * s.filt_w) != hipSuccess ||
                hipMalloc(&c, n_out * 4) != hipSuccess || hipMalloc(&d, n_out * 4) != hipSuccess) {
                for (float* p : {a, b, c, d})
                    if (p) hipFree(p);
                return fail(CONV2D_ENOMEM, "batch tune: device allocation");
            }
            in.push_back(a);
            f.push_back(b);
            out.push_back(c);
            ref.push_back(d);
            int rc = launch_fill_uniform(a, n_in, 1000 + k, 0, st);
            if (!rc) rc = launch_fill_uniform(b, (size_t)s.filt_h * s.filt_w, 2000 + k, 0, st);
            if (!rc) rc = launch_reference(s, a, b, d, st);
            if (rc) return rc;
        }
        CONV2D_HIP(hipStreamSynchronize(st));
        return CONV2D_OK;
    }

    // Descriptor and owner tables for a configuration's tiles.
    int layout(const conv2d_config& c)
    {
        std::vector<ConvDesc> descs(shapes.size());
        std::vector<unsigned short> owner;
        long long total = 0;
        for (size_t k = 0; k < shapes.size(); ++k) {
            const conv2d_shape& s = shapes[k];
            const Geometry geo = geometry(s.out_h, s.out_w, c);
            descs[k] = ConvDesc{in[k], f[k], out[k], s.out_h, s.out_w, geo.tiles_x, (int)total,
                                (unsigned)(4ull * (s.out_h + s.filt_h - 1) * (s.out_w + s.filt_w - 1)), geo.n_tiles};
            owner.insert(owner.end(), (size_t)geo.n_tiles, (unsigned short)k);
            total += geo.n_tiles;
        }
        if (total > INT_MAX) return fail(CONV2D_EINVAL, "batch tune: too many tiles");
        tiles = (int)total;
        if (d_owner) hipFree(d_owner);
        d_owner = nullptr;
        if (hipMalloc(&d_owner, sizeof(unsigned short) * owner.size()) != hipSuccess)
            return fail(CONV2D_ENOMEM, "batch tune: device allocation");
        CONV2D_HIP(hipMemcpy(d_desc, descs.data(), sizeof(ConvDesc) * descs.size(), hipMemcpyHostToDevice));
        CONV2D_HIP(hipMemcpy(d_owner, owner.data(), sizeof(unsigned short) * owner.size(), hipMemcpyHostToDevice));
        return CONV2D_OK;
    }

    int launch(const Module& m, const conv2d_config& c)
    {
        return launch_batch_kernel(m, c, std::max(8, tiles), d_desc, d_owner, tiles, st);
    }

    // One launch on NaN-filled outputs, then a bitwise comparison with the
    // reference; *ok tells whether every output matched.
    int verify(const Module& m, const conv2d_config& c, bool* ok)
    {
        for (size_t k = 0; k < shapes.size(); ++k) {
            int rc = launch_fill_value(out[k], (size_t)shapes[k].out_h * shapes[k].out_w, __builtin_nanf(""), st);
            if (rc) return rc;
        }
        int rc = launch(m, c);
        if (rc) return rc;
        CONV2D_HIP(hipMemsetAsync(d_count, 0, sizeof(unsigned), st));
        for (size_t k = 0; k < shapes.size() && !rc; ++k)
            rc = launch_count_mismatch(out[k], ref[k], (size_t)shapes[k].out_h * shapes[k].out_w, d_count, st);
        if (rc) return rc;
        unsigned bad = 0;
        CONV2D_HIP(hipMemcpyAsync(&bad, d_count, sizeof bad, hipMemcpyDeviceToHost, st));
        CONV2D_HIP(hipStreamSynchronize(st));
        *ok = bad == 0;
        return CONV2D_OK;
    }

    int time_sustained(const Module& m, const conv2d_config& c, int warmup, int reps, double* ms)
    {
        for (int k = 0; k < warmup; ++k) {
            int rc = launch(m, c);
            if (rc) return rc;
        }
        CONV2D_HIP(hipEventRecord(e0, st));
        for (int k = 0; k < reps; ++k) {
            int rc = launch(m, c);
            if (rc) return rc;
        }
        CONV2D_HIP(hipEventRecord(e1, st));
        CONV2D_HIP(hipEventSynchronize(e1));
        float t = 0;
        CONV2D_HIP(hipEventElapsedTime(&t, e0, e1));
        *ms = t / reps;
        return CONV2D_OK;
    }
};

}  // namespace
}  // namespace conv2d

extern "C" int conv2d_size_bucket(int out_h, int out_w) { return size_bucket(out_h, out_w); }

extern "C" void conv2d_batch_tune_defaults(conv2d_batch_tune_opts* o)
{
    if (!o) return;
    *o = conv2d_batch_tune_opts{};
    o->candidates = 12;
    o->warmup = 3;
    o->reps = 50;
    o->tie_rel = 0.005;
}

extern "C" int conv2d_batch_tune(int n, const conv2d_shape* shapes, const conv2d_batch_tune_opts* opts,
                                 conv2d_batch_tune_result* res)
{
    clear_error();
    if (!res) return fail(CONV2D_EINVAL, "res is NULL");
    *res = conv2d_batch_tune_result{};
    if (n < 1 || !shapes) return fail(CONV2D_EINVAL, "a batch needs n >= 1 shapes");
    for (int i = 0; i < n; ++i) {
        int rc = shape_check(shapes[i]);
        if (rc) return fail(rc, "problem " + std::to_string(i) + ": " + last_error_cstr());
    }
    conv2d_batch_tune_opts o;
    conv2d_batch_tune_defaults(&o);
    if (opts) o = *opts;
    o.candidates = std::max(0, o.candidates);
    o.warmup = std::max(0, o.warmup);
    o.reps = std::max(1, o.reps);
    o.tie_rel = std::max(0.0, o.tie_rel);
    DeviceInfo dev;
    int rc = current_device_info(&dev);
    if (rc) return rc;
    const std::string wp = winners_path_or_default(o.winners_path);
    const std::string rdir = (o.results_dir && *o.results_dir) ? std::string(o.results_dir) : library_dir() + "/tuned";

    // Groups: (fh, fw, bucket), bucket 0 when not tuning by size.
    std::map<std::tuple<int, int, int>, std::vector<conv2d_shape>> groups;
    for (int i = 0; i < n; ++i) {
        const int bk = o.buckets ? size_bucket(shapes[i].out_h, shapes[i].out_w) : 0;
        groups[std::make_tuple(shapes[i].filt_h, shapes[i].filt_w, bk)].push_back(shapes[i]);
    }
    res->n_groups = (int)groups.size();

    // Candidates of every group (the current choice first), compiled up front
    // on a pool of host threads.
    std::vector<std::vector<conv2d_config>> cands;
    std::vector<std::pair<conv2d_shape, conv2d_config>> to_compile;
    for (const auto& kv : groups) {
        const int fh = std::get<0>(kv.first), fw = std::get<1>(kv.first), bk = std::get<2>(kv.first);
        std::vector<conv2d_config> c{lookup_batch_config(dev, wp, fh, fw, bk)};
        for (const auto& x : sweep_candidates(dev, rdir, fh, fw, o.candidates)) {
            bool seen = false;
            for (const auto& e : c) seen = seen || config_equal(e, x);
            if (!seen) c.push_back(x);
        }
        for (const auto& x : c) to_compile.push_back({conv2d_shape{4096, 4096, fh, fw}, x});
        cands.push_back(std::move(c));
    }
    {
        const int nthreads = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
        std::atomic<size_t> next{0};
        std::vector<std::thread> pool;
        for (int t = 0; t < nthreads; ++t)
            pool.emplace_back([&] {
                for (size_t i = next++; i < to_compile.size(); i = next++)
                    (void)compile_direct(to_compile[i].first, to_compile[i].second, 1, 1, dev.arch, nullptr, nullptr,
                                         true);
            });
        for (auto& th : pool) th.join();
        clear_error();
        if (o.verbose) std::fprintf(stderr, "[batch tune] %zu candidates compiled\n", to_compile.size());
    }

    int g = 0;
    for (const auto& kv : groups) {
        const int fh = std::get<0>(kv.first), fw = std::get<1>(kv.first), bk = std::get<2>(kv.first);
        GroupBench gb;
        gb.shapes = kv.second;
        rc = gb.init();
        if (rc) return rc;
        const std::vector<conv2d_config>& cand = cands[(size_t)g];
        std::vector<RecordT<conv2d_config>> timed;
        double current_ms = -1;   // stays -1 when the current choice did not build or verify
        for (size_t k = 0; k < cand.size(); ++k) {
            conv2d_config c = cand[k];
            Module m;
            if (batch_module(dev, fh, fw, &c, &m) != CONV2D_OK) {
                clear_error();
                continue;
            }
            bool ok = false;
            rc = gb.layout(c);
            if (!rc) rc = gb.verify(m, c, &ok);
            double ms = 0;
            if (!rc && ok) rc = gb.time_sustained(m, c, o.warmup, o.reps, &ms);
            unload_module(&m);
            if (rc) return rc;
            if (!ok) continue;
            if (k == 0) current_ms = ms;
            timed.push_back(RecordT<conv2d_config>{c, kOk, ms, ms, ms, o.reps});
            if (o.verbose)
                std::fprintf(stderr, "[batch tune] %dx%d bucket %d (%zu problems) %s: %.4f ms\n", fh, fw, bk,
                             kv.second.size(), config_str(c).c_str(), ms);
        }
        if (timed.empty()) return fail(CONV2D_EVERIFY, "batch tune: no configuration ran and verified");
        std::sort(timed.begin(), timed.end(), [](const auto& a, const auto& b) {
            return a.ms != b.ms ? a.ms < b.ms : config_less(a.c, b.c);
        });
        RecordT<conv2d_config> win = timed[0];
        for (const auto& r : timed)
            if (r.ms <= timed[0].ms * (1.0 + o.tie_rel) && config_less(r.c, win.c)) win = r;
        rc = cache_store(wp, dev.arch, batch_key(fh, fw, bk), win.c, win.ms);
        if (rc) return rc;
        if (g < CONV2D_BATCH_TUNE_MAX) {
            res->filt[2 * g] = fh;
            res->filt[2 * g + 1] = fw;
            res->bucket[g] = bk;
            res->n_problems[g] = (int)kv.second.size();
            res->before[g] = cand[0];
            res->after[g] = win.c;
            res->before_ms[g] = current_ms;
            res->after_ms[g] = win.ms;
            res->n_tried[g] = (int)timed.size();
        }
        ++g;
    }
    return CONV2D_OK;
}
