// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "conv2d.h"
#include "hotspot.h"

namespace conv2d {

// ---------------------------------------------------------------- errors
// Sets the thread-local last-error text and returns `status`.
int fail(int status, const std::string& msg);
void clear_error();
const char* last_error_cstr();
// Maps a HIP error to CONV2D_EHIP with its text (prefixed by `what`).
int hip_fail(hipError_t e, const char* what);
#define CONV2D_HIP(call)                                  \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return ::conv2d::hip_fail(e_, #call); \
    } while (0)

// ---------------------------------------------------------------- misc
uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull);
uint64_t fnv1a(const std::string& s, uint64_t h = 1469598103934665603ull);
// A kernel source with its comments removed and its blanks collapsed (one
// space inside a line, no empty lines; literals kept as they are): the text
// whose hash keys tuned results, so that editing comments or layout keeps
// them valid while any change to the code does not.
std::string code_text(const std::string& source);
std::string hex64(uint64_t v);
std::string env_str(const char* name, const char* dflt = "");
// Directory that holds this shared library.
std::string library_dir();
bool make_dirs(const std::string& path);
bool write_file_atomic(const std::string& path, const void* data, size_t n);
bool read_file(const std::string& path, std::vector<char>& out);
double now_s();

// ---------------------------------------------------------------- configs
constexpr int kMaxFilter = 63;
constexpr int kMaxThreads = 1024;
constexpr int kLdsLimitGfx950 = 163840;
bool config_axes_valid(const conv2d_config& c, std::string* why);
std::string config_str(const conv2d_config& c);
bool parse_config(const std::string& s, conv2d_config* c);
// Tuple order used for tie-breaks: (bx, by, tx, ty, lds, const, unroll).
bool config_less(const conv2d_config& a, const conv2d_config& b);
bool config_equal(const conv2d_config& a, const conv2d_config& b);
int lds_bytes(int fh, int fw, const conv2d_config& c);
int shape_check(const conv2d_shape& s);

// ---------------------------------------------------------------- JIT
// Kernel source text of the tunable direct convolution (embedded at build).
const std::string& direct_source();
uint64_t direct_source_hash();
// hiprtc options for one configuration (packed FP32 disabled).
std::vector<std::string> direct_options(const conv2d_shape& s, const conv2d_config& c,
                                        int vin, int vout, const std::string& arch, bool batch = false);
// Compile a kernel source (file name `name`, e.g. "hotspot.hip") with hiprtc
// and `opts`, or read the code object cached under the hash of source,
// compiler version and options. `what` names the build in error messages.
// Returns CONV2D_OK or CONV2D_ECOMPILE. Thread safe.
int compile_program(const std::string& source, const char* name, const std::vector<std::string>& opts,
                    const std::string& what, std::vector<char>* code, std::string* path);
// Compile (or read from the disk cache) the code object for a configuration.
// Returns CONV2D_OK or CONV2D_ECOMPILE. Thread safe.
int compile_direct(const conv2d_shape& s, const conv2d_config& c, int vin, int vout,
                   const std::string& arch, std::vector<char>* code, std::string* path,
                   bool batch = false);
std::string code_cache_dir();
// Kernel source text of the hotspot stencil (embedded at build).
const std::string& hotspot_source();
// Kernel symbol of one configuration, e.g. conv2d_direct_b16x16_t4x2_l1c0u1_f17x17.
std::string direct_kernel_name(const conv2d_shape& s, const conv2d_config& c, bool batch = false);

// A loaded module with the direct kernel and its constant-filter symbol.
struct Module {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    void* const_filter = nullptr;   // device address of conv_filter (FCONST=1)
    size_t const_bytes = 0;
};
int load_module(const std::vector<char>& code, const std::string& kernel, Module* m);
// Compiles and loads a configuration. With allow_fallback, a build whose
// kernel spills to scratch (a fully or partly unrolled row loop can, for some
// alignment classes) is replaced by the rolled loop (cfg->unroll becomes 1).
int build_module(const conv2d_shape& s, conv2d_config* cfg, int vin, int vout, const std::string& arch, bool batch,
                 bool allow_fallback, Module* m);
void unload_module(Module* m);

// ---------------------------------------------------------------- device
struct DeviceInfo {
    int device = -1;
    std::string arch;       // e.g. "gfx950" (features stripped)
    int cus = 0;
    int lds_limit = 0;      // bytes per workgroup
    int clock_khz = 0;
};
int current_device_info(DeviceInfo* info);
// Checks that [p, p+bytes) lies inside one device allocation.
int check_device_range(const void* p, size_t bytes, const char* name);

// ---------------------------------------------------------------- launch
struct Geometry {
    int tiles_x = 0, tiles_y = 0, n_tiles = 0, threads = 0;
};
Geometry geometry(int out_h, int out_w, const conv2d_config& c);
// Largest number of output rows per launch so that the input band stays below
// 2^31 bytes (buffer offsets are 32-bit).
int band_rows(const conv2d_shape& s);
// Load and store vector width of every build of the direct kernel, for rows
// of any width and pointers at any dword boundary. A gfx9-family memory
// instruction of several dwords needs only dword alignment in the alignment
// mode the ROCm driver sets. A raw buffer load checks each dword against the
// buffer's size: a 4-wide load that straddles the end of the input returns
// zeros for the dwords past it, like a load wholly past it. A 4-wide store is
// issued only where all four outputs lie inside the row.
constexpr int kVec = 4;
// Launches the direct kernel of `m` over the whole shape (in bands) on stream.
int launch_direct(const Module& m, const conv2d_shape& s, const conv2d_config& c,
                  const float* d_in, const float* d_f, float* d_out, hipStream_t stream);

// ---------------------------------------------------------------- aux kernels
int launch_reference(const conv2d_shape& s, const float* d_in, const float* d_f, float* d_out,
                     hipStream_t stream);
// The hotspot step's coefficients grouped by the term they multiply
// (T' = ka*T + ky*(N + S) + kx*(W + E) + fma(cc, P, q)), computed in double
// from the caller's FP32 coefficients and rounded once; the tunable kernel
// and the reference take the same values.
struct hs_terms {
    float ka, ky, kx, cc, q;
};
hs_terms hs_fold(const hotspot_coeffs& k);
// One explicit hotspot step, one cell per thread (see hotspot.h).
int launch_hotspot_reference_step(int rows, int cols, const float* d_in, const float* d_power, float* d_out,
                                  const hs_terms& k, hipStream_t stream);
int launch_fill_uniform(float* d, size_t n, uint64_t seed, uint64_t start, hipStream_t stream);
int launch_fill_value(float* d, size_t n, float v, hipStream_t stream);
// Counts words of a and b whose bits differ; *d_count must be a device int.
int launch_count_mismatch(const float* a, const float* b, size_t n, unsigned* d_count,
                          hipStream_t stream);
int launch_flush(float* d, size_t n, hipStream_t stream);

// ---------------------------------------------------------------- batched kernels
// Mirror of the batched kernel's ConvDesc (conv2d_direct.hip, CONV_BATCH=1).
struct ConvDesc {
    const float* in;
    const float* filt;
    float* out;
    int H, W;
    int tiles_x;
    int tile_begin;
    unsigned in_bytes;
    int n_tiles;
};
static_assert(sizeof(ConvDesc) == 48, "descriptor layout must match the kernel");

// Size bucket (1..CONV2D_SIZE_BUCKETS) of a problem for the batched path.
int size_bucket(int out_h, int out_w);
// The batched kernel's configuration for filter fh x fw from the winners
// cache: size bucket `bucket`'s entry, else the whole-batch entry (bucket 0:
// the whole-batch entry, else bucket `fallback_bucket`'s), else the 4096x4096
// winner, else the default; filter through its pointer.
conv2d_config batch_config_for(const DeviceInfo& dev, int fh, int fw, int bucket, int fallback_bucket = 0);
// Compiles and loads the batched kernel of a configuration (the rolled row
// loop replaces one that spills; cfg->unroll then becomes 1).
int batch_module(const DeviceInfo& dev, int fh, int fw, conv2d_config* cfg, Module* m);
// Launches a batched kernel over `total_tiles` tiles on `grid` workgroups.
int launch_batch_kernel(const Module& m, const conv2d_config& cfg, int grid, const void* d_desc,
                        const void* d_owner, int total_tiles, hipStream_t st);

// Seeded fill of many buffers in one launch (see conv2d_fill_uniform).
struct FillDesc {
    float* p;
    unsigned long long n;
    unsigned long long seed;
    unsigned long long reserved;
};
static_assert(sizeof(FillDesc) == 32, "fill descriptor layout");
int launch_fill_uniform_batch(const FillDesc* d_desc, int n_desc, unsigned long long max_n, hipStream_t st);

// ---------------------------------------------------------------- hotspot
// hotspot_run with the library's fixed work array (see hotspot_noalloc.hip).
int hotspot_run_fixed_work(hotspot_plan_s* plan, const float* d_temp, const float* d_power, float* d_out,
                           float* work, size_t work_cells, int steps, hotspot_coeffs k, void* stream);

// ---------------------------------------------------------------- JSON lines
// Minimal flat-object JSON: string, number and number-array values.
struct JsonObj {
    std::map<std::string, std::string> str;
    std::map<std::string, double> num;
    std::map<std::string, std::vector<double>> arr;
};
std::string json_escape(const std::string& s);
bool json_parse_line(const std::string& line, JsonObj* out);
bool append_line(const std::string& path, const std::string& line);

// ---------------------------------------------------------------- winners cache
std::string winners_default_path();
int cache_lookup(const std::string& path, const std::string& arch, const conv2d_shape& s,
                 conv2d_config* c, double* ms, bool* stale = nullptr);
int cache_store(const std::string& path, const std::string& arch, const conv2d_shape& s,
                const conv2d_config& c, double ms);
// The winner for a filter size: the entry of `prefer` if cached, else the
// most recent entry of any shape with that filter size.
int cache_lookup_filter(const std::string& path, const std::string& arch, int fh, int fw,
                        const conv2d_shape& prefer, conv2d_config* c);

}  // namespace conv2d
