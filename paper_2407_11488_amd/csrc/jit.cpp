// Run-time compilation of the tunable direct-convolution kernel with hiprtc,
// an on-disk code-object cache, and module loading.
#include <hip/hiprtc.h>

#include <atomic>
#include <cstdio>
#include <fstream>
#include <mutex>
#include <set>
#include <thread>

#include "internal.h"

namespace conv2d {

#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wc23-extensions"
static const char kDirectSource[] = {
#embed "conv2d_direct.hip"
    , 0};
#pragma clang diagnostic pop

const std::string& direct_source()
{
    static const std::string s(kDirectSource);
    return s;
}

uint64_t direct_source_hash()
{
    static const uint64_t h = fnv1a(code_text(direct_source()));
    return h;
}

std::string direct_kernel_name(const conv2d_shape& s, const conv2d_config& c, bool batch)
{
    char b[128];
    std::snprintf(b, sizeof b, "conv2d_%s_b%dx%d_t%dx%d_l%dc%du%d_f%dx%d", batch ? "batch" : "direct", c.block_x,
                  c.block_y, c.tile_x, c.tile_y, c.use_lds, c.filter_in_const, c.unroll, s.filt_h, s.filt_w);
    return b;
}

std::vector<std::string> direct_options(const conv2d_shape& s, const conv2d_config& c, int vin,
                                        int vout, const std::string& arch, bool batch)
{
    auto D = [](const char* k, int v) { return std::string("-D") + k + "=" + std::to_string(v); };
    return {
        "--offload-arch=" + arch,
        "-O3",
        "-std=c++17",
        // Packed FP32 instructions are never generated (each FMA is a plain
        // v_fmac_f32 / v_fma_f32).
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        D("CONV_BX", c.block_x), D("CONV_BY", c.block_y), D("CONV_TX", c.tile_x),
        D("CONV_TY", c.tile_y), D("CONV_USE_LDS", c.use_lds), D("CONV_FCONST", c.filter_in_const),
        D("CONV_UNROLL", c.unroll), D("CONV_FH", s.filt_h), D("CONV_FW", s.filt_w),
        D("CONV_VIN", vin), D("CONV_VOUT", vout),
        D("CONV_BATCH", batch ? 1 : 0),
        "-DCONV_NAME=" + direct_kernel_name(s, c, batch),
    };
}

std::string code_cache_dir()
{
    std::string d = env_str("CONV2D_CACHE_DIR");
    if (d.empty()) d = library_dir() + "/_cache";
    return d;
}

static std::string hiprtc_version_str()
{
    int maj = 0, min = 0;
    hiprtcVersion(&maj, &min);
    return std::to_string(maj) + "." + std::to_string(min);
}

// The cache file of a program: keyed by the hash of its source, the
// compiler version and its options.
static std::string cache_file_for(const std::string& source, const char* name, const std::vector<std::string>& opts)
{
    uint64_t h = fnv1a(source);
    h = fnv1a(hiprtc_version_str(), h);
    for (const auto& o : opts) h = fnv1a(o + "\x1f", h);
    std::string stem(name);
    stem = stem.substr(0, stem.find('.'));
    return code_cache_dir() + "/" + stem + "_" + hex64(h) + ".co";
}

// With CONV2D_COMPILE_LOG set, every distinct program a process asks for
// (hit or miss) is appended to that file as one line: the program's file
// name, then its options, separated by single spaces. conv2d_warm_cache
// replays such a list into the code-object cache.
static void log_compile_request(const char* name, const std::vector<std::string>& opts)
{
    static const std::string log = env_str("CONV2D_COMPILE_LOG");
    if (log.empty()) return;
    std::string line(name);
    for (const auto& o : opts) {
        if (o.empty() || o.find_first_of(" \t\n") != std::string::npos) return;  // not representable
        line += " " + o;
    }
    static std::mutex mu;
    static std::set<std::string> seen;
    std::lock_guard<std::mutex> lock(mu);
    if (seen.insert(line).second) append_line(log, line);
}

int compile_program(const std::string& source, const char* name, const std::vector<std::string>& opts,
                    const std::string& what, std::vector<char>* code, std::string* path)
{
    log_compile_request(name, opts);
    const std::string dir = code_cache_dir();
    const std::string file = cache_file_for(source, name, opts);
    if (path) *path = file;
    std::vector<char> cached;
    if (read_file(file, cached) && cached.size() > 64) {
        if (code) code->swap(cached);
        return CONV2D_OK;
    }

    hiprtcProgram prog = nullptr;
    if (hiprtcCreateProgram(&prog, source.c_str(), name, 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS)
        return fail(CONV2D_ECOMPILE, "hiprtcCreateProgram failed");
    std::vector<const char*> argv;
    for (const auto& o : opts) argv.push_back(o.c_str());
    hiprtcResult r = hiprtcCompileProgram(prog, (int)argv.size(), argv.data());
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n + 1, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return fail(CONV2D_ECOMPILE, what + ": " + log.c_str());
    }
    size_t n = 0;
    hiprtcGetCodeSize(prog, &n);
    std::vector<char> obj(n);
    hiprtcGetCode(prog, obj.data());
    hiprtcDestroyProgram(&prog);
    if (make_dirs(dir)) write_file_atomic(file, obj.data(), obj.size());  // best effort
    if (code) code->swap(obj);
    return CONV2D_OK;
}

int compile_direct(const conv2d_shape& s, const conv2d_config& c, int vin, int vout,
                   const std::string& arch, std::vector<char>* code, std::string* path, bool batch)
{
    return compile_program(direct_source(), "conv2d_direct.hip", direct_options(s, c, vin, vout, arch, batch),
                           "config " + config_str(c), code, path);
}

int load_module(const std::vector<char>& code, const std::string& kernel, Module* m)
{
    *m = Module{};
    CONV2D_HIP(hipModuleLoadData(&m->mod, code.data()));
    hipError_t e = hipModuleGetFunction(&m->fn, m->mod, kernel.c_str());
    if (e != hipSuccess) {
        hipModuleUnload(m->mod);
        m->mod = nullptr;
        return hip_fail(e, ("hipModuleGetFunction(" + kernel + ")").c_str());
    }
    hipDeviceptr_t p = nullptr;
    size_t bytes = 0;
    if (hipModuleGetGlobal(&p, &bytes, m->mod, "conv_filter") == hipSuccess) {
        m->const_filter = p;
        m->const_bytes = bytes;
    } else {
        (void)hipGetLastError();
    }
    return CONV2D_OK;
}

int build_module(const conv2d_shape& s, conv2d_config* cfg, int vin, int vout, const std::string& arch, bool batch,
                 bool allow_fallback, Module* m)
{
    for (int attempt = 0; attempt < 2; ++attempt) {
        std::vector<char> code;
        int rc = compile_direct(s, *cfg, vin, vout, arch, &code, nullptr, batch);
        if (rc) return rc;
        rc = load_module(code, direct_kernel_name(s, *cfg, batch), m);
        if (rc) return rc;
        if (!allow_fallback || cfg->unroll == 1) return CONV2D_OK;
        int scratch = 0;
        if (hipFuncGetAttribute(&scratch, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, m->fn) != hipSuccess) {
            (void)hipGetLastError();
            return CONV2D_OK;
        }
        if (scratch == 0) return CONV2D_OK;
        unload_module(m);
        cfg->unroll = 1;
    }
    return CONV2D_OK;
}

void unload_module(Module* m)
{
    if (m && m->mod) hipModuleUnload(m->mod);
    if (m) *m = Module{};
}

}  // namespace conv2d

extern "C" int conv2d_warm_cache(const char* manifest, int threads, int* n_compiled, int* n_cached)
{
    using namespace conv2d;
    clear_error();
    if (n_compiled) *n_compiled = 0;
    if (n_cached) *n_cached = 0;
    if (!manifest) return fail(CONV2D_EINVAL, "manifest is NULL");
    std::ifstream in(manifest);
    if (!in) return fail(CONV2D_EINVAL, std::string("cannot read ") + manifest);
    struct Job {
        std::string name;
        std::vector<std::string> opts;
    };
    std::vector<Job> jobs;
    std::set<std::string> seen;
    std::string line;
    while (std::getline(in, line)) {
        if (line.empty() || line[0] == '#' || !seen.insert(line).second) continue;
        Job j;
        size_t p = 0;
        while (p < line.size()) {
            size_t q = line.find(' ', p);
            if (q == std::string::npos) q = line.size();
            if (q > p) (j.name.empty() ? j.name : (j.opts.push_back(""), j.opts.back())) = line.substr(p, q - p);
            p = q + 1;
        }
        if (j.name != "conv2d_direct.hip" && j.name != "hotspot.hip")
            return fail(CONV2D_EINVAL, "unknown program in manifest: " + j.name);
        jobs.push_back(std::move(j));
    }
    if (threads <= 0) threads = (int)std::thread::hardware_concurrency();
    threads = std::max(1, std::min(threads, 64));
    std::atomic<size_t> next{0};
    std::atomic<int> compiled{0}, cached{0}, failed{0};
    std::mutex err_mu;
    std::string first_err;
    auto work = [&]() {
        for (size_t k = next++; k < jobs.size(); k = next++) {
            const Job& j = jobs[k];
            const std::string& src = j.name == "hotspot.hip" ? hotspot_source() : direct_source();
            std::vector<char> probe;
            if (read_file(cache_file_for(src, j.name.c_str(), j.opts), probe) && probe.size() > 64) {
                ++cached;
                continue;
            }
            if (compile_program(src, j.name.c_str(), j.opts, "manifest entry", nullptr, nullptr) == CONV2D_OK) {
                ++compiled;
            } else {
                ++failed;
                std::lock_guard<std::mutex> lock(err_mu);
                if (first_err.empty()) first_err = last_error_cstr();
            }
        }
    };
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t) pool.emplace_back(work);
    for (auto& t : pool) t.join();
    if (n_compiled) *n_compiled = compiled;
    if (n_cached) *n_cached = cached;
    if (failed) return fail(CONV2D_ECOMPILE, std::to_string(failed.load()) + " manifest entries failed: " + first_err);
    return CONV2D_OK;
}
