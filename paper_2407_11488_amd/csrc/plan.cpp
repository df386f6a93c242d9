// Plain path: configuration legality, launch geometry, plans and runs.
#include <algorithm>
#include <climits>
#include <cstring>
#include <memory>
#include <mutex>

#include "internal.h"

namespace conv2d {

// ---------------------------------------------------------------- device

int current_device_info(DeviceInfo* info)
{
    static std::mutex mu;
    static std::map<int, DeviceInfo> cache;
    int dev = 0;
    CONV2D_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it == cache.end()) {
        hipDeviceProp_t p;
        CONV2D_HIP(hipGetDeviceProperties(&p, dev));
        DeviceInfo d;
        d.device = dev;
        d.arch = p.gcnArchName;
        size_t colon = d.arch.find(':');
        if (colon != std::string::npos) d.arch = d.arch.substr(0, colon);
        d.cus = p.multiProcessorCount;
        d.lds_limit = (int)p.sharedMemPerBlock;
        d.clock_khz = p.clockRate;
        it = cache.emplace(dev, d).first;
    }
    *info = it->second;
    return CONV2D_OK;
}

int check_device_range(const void* p, size_t bytes, const char* name)
{
    if (!p) return fail(CONV2D_EINVAL, std::string(name) + " is NULL");
    if (reinterpret_cast<uintptr_t>(p) % 4 != 0)
        return fail(CONV2D_EINVAL, std::string(name) + " is not 4-byte aligned");
    if (env_str("CONV2D_NO_PTR_CHECK") == "1") return CONV2D_OK;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    hipError_t e = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
    if (e != hipSuccess || !base) {
        (void)hipGetLastError();
        return fail(CONV2D_EINVAL, std::string(name) + " is not inside a device allocation");
    }
    const uintptr_t b = reinterpret_cast<uintptr_t>(base), q = reinterpret_cast<uintptr_t>(p);
    if (q < b || q + bytes > b + size)
        return fail(CONV2D_EINVAL, std::string(name) + " allocation is smaller than the shape needs (" +
                                       std::to_string(bytes) + " bytes)");
    return CONV2D_OK;
}

// ---------------------------------------------------------------- geometry

Geometry geometry(int out_h, int out_w, const conv2d_config& c)
{
    Geometry g;
    const int tw = c.block_x * c.tile_x, th = c.block_y * c.tile_y;
    g.tiles_x = (out_w + tw - 1) / tw;
    g.tiles_y = (out_h + th - 1) / th;
    g.n_tiles = g.tiles_x * g.tiles_y;
    g.threads = c.block_x * c.block_y;
    return g;
}

int band_rows(const conv2d_shape& s)
{
    const long long pitch_bytes = 4ll * ((long long)s.out_w + s.filt_w - 1);
    long long rows = (long long)INT_MAX / pitch_bytes - (s.filt_h - 1);
    if (rows < 1) rows = 1;
    return (int)std::min<long long>(rows, s.out_h);
}

int launch_direct(const Module& m, const conv2d_shape& s, const conv2d_config& c, const float* d_in,
                  const float* d_f, float* d_out, hipStream_t stream)
{
    const long long P = (long long)s.out_w + s.filt_w - 1;
    const int rows = band_rows(s);
    for (int y0 = 0; y0 < s.out_h; y0 += rows) {
        int H = std::min(rows, s.out_h - y0);
        int W = s.out_w;
        Geometry g = geometry(H, W, c);
        const float* bin = d_in + (size_t)y0 * (size_t)P;
        float* bout = d_out + (size_t)y0 * (size_t)W;
        unsigned in_bytes = (unsigned)((size_t)(H + s.filt_h - 1) * (size_t)P * 4u);
        int tiles_x = g.tiles_x, n_tiles = g.n_tiles;
        void* args[] = {&bin, &d_f, &bout, &H, &W, &tiles_x, &n_tiles, &in_bytes};
        hipError_t e = hipModuleLaunchKernel(m.fn, (unsigned)n_tiles, 1, 1, (unsigned)g.threads, 1, 1,
                                             0, stream, args, nullptr);
        if (e != hipSuccess) return fail(CONV2D_ELAUNCH, std::string("hipModuleLaunchKernel: ") +
                                                             hipGetErrorString(e));
    }
    return CONV2D_OK;
}

}  // namespace conv2d

using namespace conv2d;

// ---------------------------------------------------------------- plan object

struct conv2d_plan_s {
    int device = -1;
    std::string arch;
    conv2d_shape shape{};
    conv2d_config cfg{};
    int source = 0;          // 0 default, 1 tuned, 2 forced/given, 3 tuned on an older kernel
    Module main;
};

// ---------------------------------------------------------------- host-only API

extern "C" int conv2d_version(void) { return 100; }

extern "C" void conv2d_default_config(conv2d_config* cfg)
{
    if (cfg) *cfg = conv2d_config{16, 16, 1, 1, 1, 1, 1};
}

extern "C" int conv2d_lds_bytes(int filt_h, int filt_w, const conv2d_config* cfg)
{
    if (!cfg) return fail(CONV2D_EINVAL, "cfg is NULL");
    return lds_bytes(filt_h, filt_w, *cfg);
}

extern "C" int conv2d_config_check(conv2d_shape s, const conv2d_config* cfg, int lds_limit)
{
    clear_error();
    if (!cfg) return fail(CONV2D_EINVAL, "cfg is NULL");
    int rc = shape_check(s);
    if (rc) return rc;
    std::string why;
    if (!config_axes_valid(*cfg, &why)) return fail(CONV2D_EINVAL, why);
    const int limit = lds_limit > 0 ? lds_limit : kLdsLimitGfx950;
    const int lds = lds_bytes(s.filt_h, s.filt_w, *cfg);
    if (lds > limit)
        return fail(CONV2D_EINVAL, "LDS tile of " + std::to_string(lds) + " bytes exceeds " +
                                       std::to_string(limit));
    return CONV2D_OK;
}

extern "C" int conv2d_space(conv2d_shape s, int unroll, int lds_limit, conv2d_config* out, int cap)
{
    clear_error();
    int rc = shape_check(s);
    if (rc) return rc;
    int n = 0;
    for (int bx : {16, 32, 64, 128})
        for (int by : {1, 2, 4, 8, 16})
            for (int tx : {1, 2, 4, 8})
                for (int ty : {1, 2, 4, 8})
                    for (int lds : {0, 1})
                        for (int fc : {0, 1}) {
                            conv2d_config c{bx, by, tx, ty, lds, fc, unroll};
                            if (bx * by > kMaxThreads) continue;
                            if (lds_limit >= 0) {
                                const int lim = lds_limit > 0 ? lds_limit : kLdsLimitGfx950;
                                if (lds_bytes(s.filt_h, s.filt_w, c) > lim) continue;
                            }
                            if (out && n < cap) out[n] = c;
                            ++n;
                        }
    return n;
}

extern "C" int conv2d_compile(conv2d_shape s, const conv2d_config* cfg, int vec_in, int vec_out,
                              char* path_out, int path_cap)
{
    clear_error();
    int rc = conv2d_config_check(s, cfg, 0);
    if (rc) return rc;
    auto ok_vec = [](int v) { return v == 1 || v == 2 || v == 4; };
    if (!ok_vec(vec_in) || !ok_vec(vec_out)) return fail(CONV2D_EINVAL, "vector widths must be 1, 2 or 4");
    std::string path;
    rc = compile_direct(s, *cfg, vec_in, vec_out, env_str("CONV2D_ARCH", "gfx950"), nullptr, &path);
    if (rc) return rc;
    if (path_out && path_cap > 0) {
        std::strncpy(path_out, path.c_str(), (size_t)path_cap - 1);
        path_out[path_cap - 1] = '\0';
    }
    return CONV2D_OK;
}

extern "C" int conv2d_geometry(conv2d_shape s, const conv2d_config* cfg, int* tiles_x, int* tiles_y,
                               int* threads)
{
    clear_error();
    if (!cfg) return fail(CONV2D_EINVAL, "cfg is NULL");
    int rc = shape_check(s);
    if (rc) return rc;
    std::string why;
    if (!config_axes_valid(*cfg, &why)) return fail(CONV2D_EINVAL, why);
    Geometry g = geometry(std::min(s.out_h, band_rows(s)), s.out_w, *cfg);
    if (tiles_x) *tiles_x = g.tiles_x;
    if (tiles_y) *tiles_y = g.tiles_y;
    if (threads) *threads = g.threads;
    return CONV2D_OK;
}

// ---------------------------------------------------------------- plan / run

// Builds the plan's module. A configuration the library chose (tuned or
// default) falls back to the rolled row loop if it spills; a given or forced
// one is built as asked. Only the unroll can change, which does not affect
// the launch geometry.
static int build_module(conv2d_plan_s* p)
{
    conv2d_config c = p->cfg;
    int rc = build_module(p->shape, &c, kVec, kVec, p->arch, false, p->source != 2, &p->main);
    if (rc == CONV2D_OK) p->cfg = c;
    return rc;
}

extern "C" int conv2d_plan(conv2d_plan_t* plan, conv2d_shape s, const conv2d_config* cfg)
{
    clear_error();
    if (!plan) return fail(CONV2D_EINVAL, "plan is NULL");
    *plan = nullptr;
    int rc = shape_check(s);
    if (rc) return rc;
    DeviceInfo dev;
    rc = current_device_info(&dev);
    if (rc) return rc;

    auto p = std::make_unique<conv2d_plan_s>();
    p->device = dev.device;
    p->arch = dev.arch;
    p->shape = s;
    const std::string forced = env_str("CONV2D_FORCE_CONFIG");
    if (!forced.empty()) {
        if (!parse_config(forced, &p->cfg))
            return fail(CONV2D_EINVAL, "CONV2D_FORCE_CONFIG is not bx,by,tx,ty,lds,const[,unroll]");
        p->source = 2;
    } else if (cfg) {
        p->cfg = *cfg;
        p->source = 2;
    } else {
        double ms = 0;
        std::string wp = env_str("CONV2D_WINNERS");
        if (wp.empty()) wp = winners_default_path();
        bool stale = false;
        if (cache_lookup(wp, dev.arch, s, &p->cfg, &ms, &stale) == CONV2D_OK) {
            p->source = stale ? 3 : 1;
        } else if (cache_lookup_filter(wp, dev.arch, s.filt_h, s.filt_w, conv2d_shape{4096, 4096, s.filt_h, s.filt_w},
                                       &p->cfg) == CONV2D_OK &&
                   conv2d_config_check(s, &p->cfg, dev.lds_limit) == CONV2D_OK) {
            // No entry for this shape: the same filter's winner for another
            // shape (4096 x 4096 first) usually beats the default by far.
            p->source = 4;
        } else {
            conv2d_default_config(&p->cfg);
            p->source = 0;
        }
        clear_error();
    }
    rc = conv2d_config_check(s, &p->cfg, dev.lds_limit);
    if (rc) return rc;
    rc = build_module(p.get());
    if (rc) return rc;
    *plan = p.release();
    return CONV2D_OK;
}

extern "C" int conv2d_plan_config(conv2d_plan_t plan, conv2d_config* cfg, int* tuned)
{
    clear_error();
    if (!plan) return fail(CONV2D_EINVAL, "plan is NULL");
    if (cfg) *cfg = plan->cfg;
    if (tuned) *tuned = plan->source;
    return CONV2D_OK;
}

static int check_buffers(const conv2d_shape& s, const float* d_in, const float* d_f, const float* d_out)
{
    const size_t in_bytes = 4ull * ((size_t)s.out_h + s.filt_h - 1) * ((size_t)s.out_w + s.filt_w - 1);
    const size_t f_bytes = 4ull * (size_t)s.filt_h * s.filt_w;
    const size_t out_bytes = 4ull * (size_t)s.out_h * s.out_w;
    int rc = check_device_range(d_in, in_bytes, "d_in");
    if (!rc) rc = check_device_range(d_f, f_bytes, "d_filter");
    if (!rc) rc = check_device_range(d_out, out_bytes, "d_out");
    if (rc) return rc;
    auto overlap = [](const void* a, size_t na, const void* b, size_t nb) {
        uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
        return x < y + nb && y < x + na;
    };
    if (overlap(d_out, out_bytes, d_in, in_bytes) || overlap(d_out, out_bytes, d_f, f_bytes))
        return fail(CONV2D_EINVAL, "d_out overlaps d_in or d_filter");
    return CONV2D_OK;
}

extern "C" int conv2d_run(conv2d_plan_t plan, const float* d_in, const float* d_filter, float* d_out,
                          void* stream)
{
    clear_error();
    if (!plan) return fail(CONV2D_EINVAL, "plan is NULL");
    int dev = -1;
    CONV2D_HIP(hipGetDevice(&dev));
    if (dev != plan->device) return fail(CONV2D_EINVAL, "plan was made for another device");
    int rc = check_buffers(plan->shape, d_in, d_filter, d_out);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);

    const Module* m = &plan->main;   // pointers are dword aligned (check_buffers)
    if (plan->cfg.filter_in_const) {
        if (!m->const_filter || m->const_bytes < sizeof(float) * plan->shape.filt_h * plan->shape.filt_w)
            return fail(CONV2D_EHIP, "module has no conv_filter symbol of the filter's size");
        CONV2D_HIP(hipMemcpyAsync(m->const_filter, d_filter,
                                  sizeof(float) * plan->shape.filt_h * plan->shape.filt_w,
                                  hipMemcpyDeviceToDevice, st));
    }
    return launch_direct(*m, plan->shape, plan->cfg, d_in, d_filter, d_out, st);
}

extern "C" void conv2d_destroy(conv2d_plan_t plan)
{
    if (!plan) return;
    unload_module(&plan->main);
    delete plan;
}

extern "C" int conv2d_reference(conv2d_shape s, const float* d_in, const float* d_filter, float* d_out,
                                void* stream)
{
    clear_error();
    int rc = shape_check(s);
    if (rc) return rc;
    rc = check_buffers(s, d_in, d_filter, d_out);
    if (rc) return rc;
    return launch_reference(s, d_in, d_filter, d_out, static_cast<hipStream_t>(stream));
}

extern "C" int conv2d_fill_uniform(float* d_out, size_t n, uint64_t seed, uint64_t start, void* stream)
{
    clear_error();
    int rc = check_device_range(d_out, n * sizeof(float), "d_out");
    if (rc) return rc;
    return launch_fill_uniform(d_out, n, seed, start, static_cast<hipStream_t>(stream));
}

extern "C" const char* conv2d_last_error(void)
{
    return conv2d::last_error_cstr();
}

extern "C" const char* conv2d_kernel_hash(void)
{
    static const std::string h = hex64(direct_source_hash());
    return h.c_str();
}
