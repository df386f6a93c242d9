/*
 * conv2d.h — C ABI of the MI355X (gfx950) auto-tuned direct 2D convolution.
 *
 * The operation (the convolution benchmark of the paper's Section 5, whose
 * tunable parameters are Table 1; the paper names the kernel, the formula
 * below is the valid cross-correlation that kernel computes):
 *
 *     out[y][x] = sum_{i<fh} sum_{j<fw} in[y+i][x+j] * f[i][j]
 *
 * for 0 <= y < out_h, 0 <= x < out_w. `in` is (out_h+fh-1) x (out_w+fw-1),
 * `f` is fh x fw and `out` is out_h x out_w, all dense row-major FP32 (row
 * pitch = row width). No filter flip, no implicit padding: the caller's input
 * already holds the halo.
 *
 * Conventions for every entry point:
 *  - Return 0 (CONV2D_OK) on success or a negative conv2d_status; nothing
 *    throws across this boundary. conv2d_last_error() returns a thread-local
 *    message for the last non-zero return on the calling thread.
 *  - d_* pointers are device memory on the current HIP device, owned by the
 *    caller; the library never frees them. They must be 4-byte aligned, and
 *    `d_out` must not overlap `d_in` or `d_filter`. Pointers are checked
 *    against their allocation (hipMemGetAddressRange) before any launch, so a
 *    buffer that is too small is an error (CONV2D_EINVAL), not a fault.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *    null stream). The caller keeps the buffers alive until the stream has
 *    passed the call.
 *  - Every configuration accumulates each output in one FP32 register, with
 *    fused multiply-add, taps in i-ascending then j-ascending order, starting
 *    from 0. Results are therefore bitwise identical across configurations,
 *    batch and serving paths, and the reference kernel.
 *  - Filter sizes are limited to 1..63 per axis; out_h, out_w >= 1.
 */
#ifndef CONV2D_H
#define CONV2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum conv2d_status {
    CONV2D_OK = 0,
    CONV2D_EINVAL = -1,    /* bad argument, shape, config or pointer */
    CONV2D_ENOMEM = -2,    /* device or host allocation failed */
    CONV2D_ECOMPILE = -3,  /* hiprtc rejected the configuration */
    CONV2D_ELAUNCH = -4,   /* the kernel launch failed */
    CONV2D_ENOTUNED = -5,  /* no tuned winner for this shape and none forced */
    CONV2D_EVERIFY = -6,   /* a configuration's output differed from the reference */
    CONV2D_EHIP = -7,      /* another HIP runtime error (message in last_error) */
    CONV2D_EBUSY = -8      /* serving: request cannot be admitted now */
} conv2d_status;

/* One point of the search space (the MI355X version of the paper's Table 1
 * convolution parameters). */
typedef struct conv2d_config {
    int block_x;          /* threads along x: 16, 32, 64, 128 (block_size_x) */
    int block_y;          /* threads along y: 1, 2, 4, 8, 16 (block_size_y) */
    int tile_x;           /* outputs per thread along x: 1, 2, 4, 8 (tile_size_x) */
    int tile_y;           /* outputs per thread along y: 1, 2, 4, 8 (tile_size_y) */
    int use_lds;          /* 1: stage the workgroup's input halo in LDS (use_shmem) */
    int filter_in_const;  /* 1: filter in a __constant__ array, 0: const global pointer
                             (the analogue of read_only) */
    int unroll;           /* input-row loop unroll: 1, 2, 4, or 0 = full
                             (the paper's tunable partial unroll, Section 3) */
} conv2d_config;

typedef struct conv2d_shape {
    int out_h, out_w;     /* output rows and columns */
    int filt_h, filt_w;   /* filter rows and columns (input is (out_h+filt_h-1) x (out_w+filt_w-1)) */
} conv2d_shape;

typedef struct conv2d_plan_s *conv2d_plan_t;
typedef struct conv2d_batch_s *conv2d_batch_t;

/* ---------------------------------------------------------------- host only
 * These never touch a GPU and can be called on a machine without one. */

/* Library version (major*10000 + minor*100 + patch).
 * Source: none in the paper (library metadata). */
int conv2d_version(void);

/* Thread-local text of the last non-zero return on this thread ("" if none).
 * Source: none in the paper (this ABI's error reporting). */
const char *conv2d_last_error(void);

/* Hex hash of the tunable kernel source built into this library, taken over
 * its code with comments and blank runs removed (keys the winners cache and
 * the tuner's results; editing comments keeps them valid). Static storage,
 * never NULL.
 * Source: none in the paper (the key under which this library stores what
 * the Section 3 measurements found). */
const char *conv2d_kernel_hash(void);

/* The untuned default configuration: the textbook 16x16-thread tiled kernel,
 * one output per thread, LDS halo, filter in constant memory, unroll 1.
 * Source: Section 4 measures tuning against the space's median; this fixed
 * point of the Table 1 space is the library's second baseline (tuned/default). */
void conv2d_default_config(conv2d_config *cfg);

/* LDS bytes a configuration needs for a filter size (0 when use_lds = 0).
 * Source: Table 1 (use_shmem: the input halo staged in shared memory). */
int conv2d_lds_bytes(int filt_h, int filt_w, const conv2d_config *cfg);

/* Legality of a configuration for a shape: axis values in range,
 * block_x*block_y <= 1024, LDS bytes <= lds_limit (pass 0 for the gfx950
 * value, 163840). Returns CONV2D_OK or CONV2D_EINVAL with a reason.
 * Source: Table 1 (the parameter values); the paper does not print its
 * restrictions, only the restricted space's size (Table 3). */
int conv2d_config_check(conv2d_shape s, const conv2d_config *cfg, int lds_limit);

/* Enumerates the restricted search space for a shape in axis order
 * (block_x, block_y, tile_x, tile_y, use_lds, filter_in_const), with the given
 * unroll for every point; writes up to `cap` configurations to `out` (may be
 * NULL) and returns the number of legal points (or a negative status).
 * With lds_limit < 0 only the thread-count restriction is applied.
 * Source: Table 1 (the convolution's tunable parameters) and Table 3 (the
 * search-space size row). */
int conv2d_space(conv2d_shape s, int unroll, int lds_limit, conv2d_config *out, int cap);

/* Compiles one configuration for gfx950 with hiprtc into the code-object
 * cache (no GPU needed). vec_in/vec_out are the load and store vector widths
 * 1, 2 or 4; plans, the tuner and the batched path build with 4 and 4 for
 * rows of any width (an access of several dwords needs only dword alignment
 * on gfx950, and each dword of a buffer load is range-checked).
 * Writes the cache file path to path_out (if non-NULL, cap bytes).
 * Returns CONV2D_OK or CONV2D_ECOMPILE (log in last_error).
 * Source: Section 3 (each configuration is compiled before it is benchmarked). */
int conv2d_compile(conv2d_shape s, const conv2d_config *cfg, int vec_in, int vec_out,
                   char *path_out, int path_cap);

/* Fills the code-object cache from a manifest: a text file with one program
 * per line (its file name, conv2d_direct.hip or hotspot.hip, then its hiprtc
 * options, separated by spaces; '#' starts a comment line), as a process
 * writes it to the file named by the environment variable CONV2D_COMPILE_LOG.
 * Compiles each program not yet cached on up to `threads` host threads (0:
 * all), no GPU needed, so that a later run on a GPU compiles nothing.
 * *n_compiled and *n_cached (may be NULL) receive the counts. Returns
 * CONV2D_OK, CONV2D_EINVAL (unreadable file, unknown program) or
 * CONV2D_ECOMPILE (entries that failed; the first log in last_error).
 * Source: none in the paper (a build step of this library). */
int conv2d_warm_cache(const char *manifest, int threads, int *n_compiled, int *n_cached);

/* Launch geometry of a configuration: tiles along x and y for one band of
 * rows (the kernel covers the output with tiles of
 * (block_x*tile_x) x (block_y*tile_y), one workgroup per tile).
 * Source: Table 1 (block_size_x/y threads, tile_size_x/y outputs per thread). */
int conv2d_geometry(conv2d_shape s, const conv2d_config *cfg, int *tiles_x, int *tiles_y,
                    int *threads_per_block);

/* Winners cache (JSON lines; the last line for a key wins). Key: GPU arch,
 * shape, and the kernel source hash. arch may be NULL for the current
 * device's arch. lookup returns CONV2D_ENOTUNED when absent.
 * Source: Section 6 (one tuned configuration per kernel and device, Tables
 * 4-5); the file format is this library's. */
int conv2d_cache_lookup(const char *path, const char *arch, conv2d_shape s,
                        conv2d_config *cfg, double *ms);
int conv2d_cache_store(const char *path, const char *arch, conv2d_shape s,
                       const conv2d_config *cfg, double ms);

/* ---------------------------------------------------------------- plain path */

/* Creates a plan for one shape on the current device. cfg = NULL takes the
 * tuned winner for this shape from the winners cache (env CONV2D_WINNERS,
 * else the tuned/winners.jsonl file beside this library), else the winner of
 * the same filter size for another shape (4096 x 4096 first, else the most
 * recent) when it is legal for this shape, else the default
 * configuration; the environment variable CONV2D_FORCE_CONFIG
 * ("bx,by,tx,ty,lds,const,unroll") overrides both. Compiles (or loads from the
 * code-object cache) and loads the module. The plan owns the module.
 * Source: Section 5 (the convolution benchmark kernel) with a point of the
 * Table 1 space; the formula is the one at the top of this header. */
int conv2d_plan(conv2d_plan_t *plan, conv2d_shape s, const conv2d_config *cfg);

/* The configuration a plan uses, and whether it came from the winners cache
 * (*tuned = 1; 3 when that entry was tuned with an older revision of the
 * kernel source; 4 when it is the same filter's winner for another shape),
 * was forced or given (2), or is the default (0).
 * Source: Table 1 (the parameters of the configuration). */
int conv2d_plan_config(conv2d_plan_t plan, conv2d_config *cfg, int *tuned);

/* Enqueues one convolution on `stream`. With filter_in_const = 1 the filter is
 * first copied (device to device, on the same stream) into the module's
 * constant array: such a plan must not run concurrently on two streams. The
 * call may be recorded by stream capture into a graph (a copy node, when the
 * filter goes to constant memory, then the kernel node); replays read the
 * buffers' current contents. Pointers need 4-byte alignment only (one module
 * serves every alignment).
 * Source: Section 5 (the convolution benchmark kernel); Table 1 (read_only,
 * use_shmem, tile and block sizes select the variant enqueued). */
int conv2d_run(conv2d_plan_t plan, const float *d_in, const float *d_filter, float *d_out,
               void *stream);

/* Frees the plan and unloads its code objects. It does not wait:
 * the caller first makes sure that no launch of the plan is queued or
 * running (synchronize the streams it ran on) and that no graph holding its
 * kernels is replayed afterwards. NULL is ignored.
 * Source: none in the paper (resource release of this ABI). */
void conv2d_destroy(conv2d_plan_t plan);

/* Plain reference kernel: one thread per output, runtime filter size, the
 * same accumulation order as every configuration. Used by the tuner to verify
 * each configuration bitwise.
 * Source: Section 5 (the convolution kernel's result, computed without
 * tiling); the tuner checks results before timing them (Section 3). */
int conv2d_reference(conv2d_shape s, const float *d_in, const float *d_filter, float *d_out,
                     void *stream);

/* Fills n floats of device memory with the seeded uniform values of the
 * splitmix64 recipe (hash element start+k of `seed`, mapped to
 * (top24 - 2^23) * 2^-23), on `stream`.
 * Source: none in the paper (synthetic inputs; the paper's inputs are in its
 * unavailable companion repository, Section 5). */
int conv2d_fill_uniform(float *d_out, size_t n, uint64_t seed, uint64_t start, void *stream);

/* ---------------------------------------------------------------- batched path
 *
 * Many convolutions of uneven sizes in one hipGraph launch (not part of the
 * paper: the batching extension of its convolution kernel). Each problem
 * gets a tuned configuration for its filter size: the batched path's own
 * whole-batch entry (0, 0, fh, fw) from conv2d_batch_tune, else its size
 * bucket's entry (0, b, fh, fw) (with CONV2D_BATCH_BY_SIZE the other way
 * round), else the winners cache entry for 4096x4096 with that filter, else
 * the most recent entry with that filter, else the default; the filter is
 * always read through its pointer. The problems sharing a filter size and
 * configuration form a group, run as one kernel over the group's tiles (a
 * workgroup per tile, the tiles of each image in row order, XCD-contiguous
 * runs). The
 * groups are parallel branches of one graph captured at plan time. Results
 * are bitwise identical to conv2d_run / conv2d_reference on the same data.
 * A batch plan must not run on two streams at once (its descriptor table is
 * shared); runs on one stream are ordered. Each input is limited to 2 GiB. */

enum {
    CONV2D_BATCH_NO_GRAPH = 1,     /* launch the group kernels directly instead of a graph */
    CONV2D_BATCH_NO_PTR_CHECK = 2, /* skip the per-problem allocation checks */
    CONV2D_BATCH_BY_SIZE = 4       /* each problem takes its size bucket's configuration */
};

/* Plans n problems (n <= 65535); shapes[i] as for conv2d_plan.
 * Source: Section 5 (the convolution kernel, applied to many problems);
 * batching is this library's extension, not the paper's. */
int conv2d_batch_plan(conv2d_batch_t *batch, int n, const conv2d_shape *shapes, int flags);

/* Enqueues all n convolutions on `stream`: d_in[i], d_f[i], d_out[i] are the
 * device buffers of problem i (host arrays of n device pointers). When the
 * pointers differ from the previous run, a 48-byte-per-problem descriptor
 * table is first copied to the device on the same stream.
 * Source: Section 5 (the convolution kernel); batching is this library's
 * extension. */
int conv2d_batch_run(conv2d_batch_t batch, const float *const *d_in, const float *const *d_f,
                     float *const *d_out, void *stream);

/* Groups of a batch: their count, the total tile count, and for the first
 * `cap` groups the filter size (filt[2g], filt[2g+1]), configuration and
 * grid size (one workgroup per tile, at least 8). Any output pointer may be
 * NULL.
 * Source: Table 1 (the configuration of each group). */
int conv2d_batch_info(conv2d_batch_t batch, int *n_groups, int *total_tiles, int *filt,
                      conv2d_config *cfgs, int *grids, int cap);

/* Frees the batch: its code objects and device buffers. It does not wait:
 * the caller first makes sure that no launch of the batch is queued or
 * running (synchronize the streams it ran on) and that no graph holding its
 * kernels is replayed afterwards. NULL is ignored.
 * Source: none in the paper (resource release of this ABI). */
void conv2d_batch_destroy(conv2d_batch_t batch);

/* Size buckets of the batched path's tuning cache, by the larger output
 * side: 1 (up to 384), 2 (385-768), 3 (769-1536), 4 (1537-3072), 5 (larger). */
#define CONV2D_SIZE_BUCKETS 5

/* The size bucket (1..CONV2D_SIZE_BUCKETS) of an out_h x out_w output
 * (host only; sides of 0 or less give bucket 1).
 * Source: none in the paper (the served workload's size classes). */
int conv2d_size_bucket(int out_h, int out_w);

/* Tunes the batched path on a batch: the problems are grouped by filter size
 * (and, with `buckets`, by size bucket too); for each group, its current
 * configuration, the `candidates` fastest points of the tuner's 4096x4096
 * sweep for that filter (results_<arch>_4096x4096_<fh>x<fw>.jsonl in
 * results_dir) and the fastest point of every workgroup tile area of that
 * sweep (filter always through its pointer) are each run as the batched
 * kernel over the group's problems (seeded data on the device), verified
 * bitwise against the reference kernel and timed with `reps` sustained
 * launches. The fastest (ties within tie_rel go to the smallest tuple) is
 * appended to the winners cache under the shape (0, 0, fh, fw), or
 * (0, b, fh, fw) for size bucket b (conv2d_batch_plan prefers the first,
 * conv2d_serve and CONV2D_BATCH_BY_SIZE plans the second). Candidates are
 * compiled on up
 * to 16 host threads first. Not part of the paper (its tuner tunes one kernel
 * on one problem); this is the batched path's own tuning.
 * Source: Section 3 (event timing of each compiled configuration) applied to
 * the batched kernel; Table 1 (the candidates' parameters). */
#define CONV2D_BATCH_TUNE_MAX 32
typedef struct conv2d_batch_tune_opts {
    const char *winners_path;  /* winners cache read and appended (NULL: $CONV2D_WINNERS or the default) */
    const char *results_dir;   /* sweep results (NULL: the tuned/ directory beside the library) */
    int candidates;            /* fastest sweep points tried per group (default 12) */
    int buckets;               /* 1: one configuration per filter size and size bucket (default 0) */
    int warmup, reps;          /* per candidate (default 3 and 50) */
    double tie_rel;            /* default 0.005 */
    int verbose;
} conv2d_batch_tune_opts;

typedef struct conv2d_batch_tune_result {
    int n_groups;                                  /* groups (the first CONV2D_BATCH_TUNE_MAX reported) */
    int filt[2 * CONV2D_BATCH_TUNE_MAX];           /* fh, fw of group g at 2g, 2g+1 */
    int bucket[CONV2D_BATCH_TUNE_MAX];             /* size bucket of group g (0: all sizes) */
    int n_problems[CONV2D_BATCH_TUNE_MAX];         /* problems of the batch in group g */
    conv2d_config before[CONV2D_BATCH_TUNE_MAX];   /* the choice before tuning */
    conv2d_config after[CONV2D_BATCH_TUNE_MAX];    /* the winner */
    double before_ms[CONV2D_BATCH_TUNE_MAX];       /* the group's kernel, sustained, ms per launch
                                                      (-1: the choice before tuning did not build or
                                                      verify, so it has no time) */
    double after_ms[CONV2D_BATCH_TUNE_MAX];
    int n_tried[CONV2D_BATCH_TUNE_MAX];            /* candidates that compiled, ran and verified */
} conv2d_batch_tune_result;

/* Source: none in the paper (option defaults). */
void conv2d_batch_tune_defaults(conv2d_batch_tune_opts *opts);
int conv2d_batch_tune(int n, const conv2d_shape *shapes, const conv2d_batch_tune_opts *opts,
                      conv2d_batch_tune_result *res);

/* Compiles the batched kernel of a configuration (filter read through its
 * pointer, 4-wide loads and stores at any dword position) for gfx950 with
 * hiprtc, no GPU needed.
 * Only s.filt_h and s.filt_w matter.
 * Source: Section 3 (compilation of each configuration). */
int conv2d_compile_batch(conv2d_shape s, const conv2d_config *cfg, char *path_out, int path_cap);

/* ---------------------------------------------------------------- serving
 *
 * A trace of requests run with continuous batching (not part of the paper:
 * the serving extension of its convolution kernel). Requests queue FIFO in
 * arrival order and are admitted while their device memory (input, filter
 * and, unless kept, output) fits `hbm_budget`; an admitted request's image
 * and filter are generated on the device from its seeds (the recipe of
 * conv2d_fill_uniform), standing in for an image that arrives in HBM. When
 * one of `streams` streams is free, every admitted request not yet launched
 * (up to max_batch) is launched as one batch: one fill launch, then one
 * batched kernel per filter size and configuration present, each request
 * taking its size bucket's configuration (as a CONV2D_BATCH_BY_SIZE batch).
 * Batches on different streams overlap on the device. A request's latency
 * runs from its arrival time to the host observing its batch's completion
 * event; outputs stay on the device. serial_plain = 1 runs the same trace one
 * request at a time through the plain kernel (the baseline). Results are
 * bitwise identical to a plain conv2d_run of the same data. */

typedef struct conv2d_request {
    double arrival_s;       /* seconds from the start of the run: finite, >= 0 and
                               non-decreasing (else CONV2D_EINVAL, before any
                               device work) */
    conv2d_shape shape;
    uint64_t seed_in;       /* image seed */
    uint64_t seed_f;        /* filter seed */
} conv2d_request;

typedef struct conv2d_serve_opts {
    size_t hbm_budget;      /* device bytes for admitted requests (default 8 GiB) */
    int streams;            /* batches in flight at once, 1..16 (default 4) */
    int max_batch;          /* requests per batch, 1..32767 (default 64) */
    int serial_plain;       /* 1: one at a time through the plain kernel */
    int keep_outputs;       /* 1: each output in its own allocation, returned in outputs[] */
} conv2d_serve_opts;

typedef struct conv2d_serve_report {
    int n_requests, n_batches;
    double wall_s;          /* first arrival to last completion */
    double req_per_s, gflops, offered_rate;
    double p50_ms, p99_ms, mean_ms, max_ms;      /* latency, nearest-rank percentiles */
    double queue_p50_ms, queue_p99_ms;           /* arrival to launch */
    double mean_batch;
    int stalled_requests;   /* requests that waited for HBM budget */
    size_t peak_bytes;      /* peak admitted bytes */
    double late_start_ms;   /* serial run: worst launch delay behind schedule */
} conv2d_serve_report;

/* Source: none in the paper (option defaults). */
void conv2d_serve_defaults(conv2d_serve_opts *opts);

/* Runs reqs[0..n) (blocking). latency_ms (may be NULL) receives each
 * request's latency; with keep_outputs, outputs[i] receives a device pointer
 * to request i's output (release with conv2d_serve_free).
 * Source: Section 5 (the convolution kernel) served to a request stream;
 * serving is this library's extension, not the paper's. */
int conv2d_serve(const conv2d_request *reqs, int n, const conv2d_serve_opts *opts,
                 conv2d_serve_report *report, double *latency_ms, float **outputs);

/* Frees outputs[0..n) returned by conv2d_serve with keep_outputs (NULL
 * entries are skipped). It does not wait for the device.
 * Source: none in the paper (resource release of this ABI). */
void conv2d_serve_free(float **outputs, int n);

/* ---------------------------------------------------------------- tuner */

typedef struct conv2d_tune_opts {
    const char *winners_path;  /* winners cache to update (NULL: none) */
    const char *results_path;  /* per-configuration results, JSON lines, resumable (NULL: none) */
    int warmup;                /* untimed launches per configuration (default 2) */
    int reps;                  /* timed launches per configuration (default 20) */
    int retime_reps;           /* sustained launches re-timing the ten fastest (default 200) */
    int flush_mall;            /* 1: overwrite a 512 MiB buffer before each timed launch */
    int threads;               /* host compile threads (0: all cores, at most 16) */
    int unroll;                /* unroll value for every point (default 1) */
    int max_configs;           /* 0: whole space, else the first N legal points (tests) */
    double tie_rel;            /* relative tie window for the winner (default 0.005) */
    int verbose;               /* 1: progress lines on stderr */
    int refine_unroll;         /* 1: also time the ten fastest points with the other unroll values */
    int strategy;              /* 0: brute force over the space (default); 1: random-restart hill
                                  climbing (one parameter one step per move; restart k starts at
                                  the idx-th unevaluated point in enumeration order,
                                  idx = splitmix64(seed, k) mod count), stopping at max_evals */
    int max_evals;             /* local search budget in evaluations (default 100) */
    uint64_t seed;             /* local search seed */
} conv2d_tune_opts;

typedef struct conv2d_tune_result {
    conv2d_config best;        /* the winner */
    double best_ms;            /* its sustained time per launch (re-timing) */
    double default_ms;         /* the default configuration's time in the winner's timing mode
                                  (sustained re-timing when retime_reps > 0, else the sweep's
                                  median); 0 if not timed. tuned/default = default_ms / best_ms */
    double median_ms;          /* time of the median-throughput configuration */
    double best_gflops, median_gflops, default_gflops;
    double impact;             /* best / median throughput of the sweep (the paper's tuning impact) */
    int n_space;               /* points in the restricted product */
    int n_illegal;             /* rejected by the shape-dependent restrictions (LDS) */
    int n_compile_fail, n_launch_fail, n_verify_fail;
    int n_timed;               /* configurations timed successfully */
    int n_resumed;             /* results reused from results_path */
    int default_rank;          /* 1-based rank of the default among timed configs (0: n/a) */
    conv2d_config top[5];      /* fastest five after re-timing, fastest first */
    double top_ms[5];
    double compile_s, measure_s; /* wall time of the compile and measure phases */
    int evaluations;           /* configurations measured in this call (failures included) */
    double best_sweep_ms;      /* the winner's time in the sweep (flushed single launches) */
    double default_sweep_ms;   /* the default's time in the sweep (0 if not timed) */
} conv2d_tune_result;

/* Defaults for every option.
 * Source: none in the paper (option defaults). */
void conv2d_tune_defaults(conv2d_tune_opts *opts);

/* Compiles every legal point (in parallel on host threads), then for each:
 * launches it once and checks its output bitwise against the reference kernel,
 * times it with HIP events (median of `reps` launches, each after a cache
 * flush), and records it. The ten fastest are re-timed with `retime_reps`
 * sustained launches (back to back, cycling through copies of the data that
 * together exceed the last-level cache); the winner is the lowest sustained
 * time, ties within tie_rel going to the smallest configuration tuple, and is
 * stored in the winners cache. Inputs are the seeded uniform recipe (input
 * seed 1, filter seed 2), on device.
 * Source: Section 3 (compile, then time each configuration with events
 * before and after the kernel; partial loop unrolling as a tunable);
 * Section 4 (tuning impact: the optimum over the median, as in Table 3);
 * Table 1 (the space). The local-search strategy is Section 4's premise
 * that a local search walks the fitness flow graph (Eq. 1). */
int conv2d_tune(conv2d_shape s, const conv2d_tune_opts *opts, conv2d_tune_result *res);

/* Times one configuration the way the tuner does: seeded inputs on the
 * device, one verified launch (bitwise against the reference kernel), then
 * `warmup` untimed and `reps` timed launches (HIP events, optional cache flush
 * before each). Writes the median and minimum milliseconds.
 * Source: Section 3 (events recorded before and after the kernel). */
int conv2d_benchmark(conv2d_shape s, const conv2d_config *cfg, int warmup, int reps, int flush_mall,
                     double *median_ms, double *min_ms);

/* The same search with a caller-supplied cost instead of the GPU (a fake
 * backend for host tests): cost(cfg, user) returns a time in ms, or a
 * negative status to mark a compile (-3), launch (-4) or verify (-6)
 * failure.
 * Source: as conv2d_tune (Sections 3-4), with the measurement replaced. */
typedef double (*conv2d_cost_fn)(const conv2d_config *cfg, void *user);
int conv2d_tune_synthetic(conv2d_shape s, conv2d_cost_fn cost, void *user,
                          const conv2d_tune_opts *opts, conv2d_tune_result *res);

#ifdef __cplusplus
}
#endif

#endif /* CONV2D_H */
