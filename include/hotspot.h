/*
 * hotspot.h — C ABI of the MI355X (gfx950) auto-tuned hotspot thermal stencil
 * with temporal tiling, the second tunable kernel of the library (the hotspot
 * kernel of the paper's Section 5, whose tunable parameters are Table 1).
 *
 * The operation: the compact thermal RC model of a chip (Huang et al.,
 * HotSpot, IEEE TVLSI 2006), advanced by explicit time steps. A rows x cols
 * grid holds each cell's temperature T and dissipated power P; one step sets
 *
 *     T'[r][c] = T + cc * ( P + (T[r-1][c] + T[r+1][c] - 2T) * gy
 *                             + (T[r][c-1] + T[r][c+1] - 2T) * gx
 *                             + (t_amb - T) * gz )
 *
 * (cc: time step over the cell's heat capacity; gx, gy: lateral conductances
 * between neighbouring cells along columns and rows; gz: conductance to the
 * ambient at t_amb). A neighbour outside the grid is the cell itself: no heat
 * crosses the chip's sides. Every step reads only the previous step's grid.
 *
 * Conventions are those of conv2d.h: 0 or a negative conv2d_status, a
 * thread-local conv2d_last_error(), caller-owned dense row-major FP32 device
 * buffers checked against their allocations, asynchronous work on `stream`.
 * Every cell is evaluated by the same FP32 expression in the same order,
 * the step's terms regrouped by what they multiply:
 *
 *     T' = a*T + ky*(N + S) + kx*(W + E) + (cc*P + q),
 *     a = 1 - cc*(2gx + 2gy + gz), ky = cc*gy, kx = cc*gx, q = cc*gz*t_amb,
 *
 * the four coefficients computed once per call in double from the given
 * FP32 ones and rounded to FP32, then s = fma(cc, P, q), x = fma(kx, W + E,
 * s), x = fma(ky, N + S, x), T' = fma(a, T, x).
 * Results are bitwise identical across configurations and
 * hotspot_reference, and within 8 n 2^-24 (max|T| + |t_amb| + n cc max|P|)
 * of the exact n steps while a >= 0 (coefficients inside the explicit step's
 * stability limit).
 */
#ifndef HOTSPOT_H
#define HOTSPOT_H

#include "conv2d.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One point of the search space (the MI355X version of Table 1's hotspot
 * parameters). */
typedef struct hotspot_config {
    int block_x;    /* threads along x: 16, 32, 64, 128, 256 (block_size_x) */
    int block_y;    /* threads along y: 1, 2, 4, 8, 16 (block_size_y) */
    int tile_x;     /* cells per thread along x: 1, 2, 4 (tile_size_x) */
    int tile_y;     /* cells per thread along y: 1, 2, 4 (tile_size_y) */
    int temporal;   /* steps per launch: 1, 2, 3, 4, 6, 8 (temporal_tiling_factor) */
    int unroll_t;   /* step loop: 1 rolled, 0 fully unrolled (loop_unroll_factor_t) */
    int sh_power;   /* 1: power kept on chip for all steps, 0: re-read every step (sh_power) */
} hotspot_config;

typedef struct hotspot_shape {
    int rows, cols;   /* grid size, each >= 1 */
} hotspot_shape;

typedef struct hotspot_coeffs {
    float cc;      /* time step over heat capacity (K per W) */
    float gx, gy;  /* lateral conductances along columns / rows (W per K) */
    float gz;      /* vertical conductance to the ambient (W per K) */
    float t_amb;   /* ambient temperature (K) */
} hotspot_coeffs;

typedef struct hotspot_plan_s *hotspot_plan_t;

/* ------------------------------------------------------------ host-only helpers */

/* Hex hash of the hotspot kernel source built into this library (its code
 * without comments and blank runs; keys the hotspot winners cache and
 * results). Static storage, never NULL.
 * Source: none in the paper (the key of this library's stored tuning results). */
const char *hotspot_kernel_hash(void);

/* (32, 8, 1, 1, 1, 1, 1): one cell per thread, one step per launch.
 * Source: Section 4 takes the median as the untuned baseline; this fixed
 * point of the Table 1 hotspot space is the library's second one. */
void hotspot_default_config(hotspot_config *cfg);

/* LDS bytes of a configuration: two buffers of the region with a one-cell
 * ring, 2 * (rows + 2) * ((cols + 2) | 1) floats.
 * Source: none in the paper (this kernel's layout; Table 1's block and tile
 * sizes and temporal_tiling_factor set the region). */
int hotspot_lds_bytes(const hotspot_config *cfg);

/* CONV2D_OK if cfg is a legal point: every value on its axis, at most 1024
 * and at least 64 threads, a region of (block_y*tile_y) x (block_x*tile_x)
 * cells larger than twice `temporal` along both axes, LDS within lds_limit
 * (<= 0: 160 KiB). Else CONV2D_EINVAL with the reason.
 * Source: Table 1 (the hotspot parameters); the paper does not print the
 * restrictions. */
int hotspot_config_check(hotspot_shape s, const hotspot_config *cfg, int lds_limit);

/* The restricted space in enumeration order (block_x, block_y, tile_x,
 * tile_y, temporal, unroll_t, sh_power, each ascending). Writes up to cap
 * entries to out (may be NULL) and returns the number of legal points, or a
 * negative status.
 * Source: Table 1 (the hotspot's tunable parameters). */
int hotspot_space(hotspot_shape s, int lds_limit, hotspot_config *out, int cap);

/* Compiles a configuration for gfx950 with hiprtc (no GPU needed); the code
 * object's path goes to path_out (cap bytes).
 * Source: Section 3 (each configuration is compiled before it is benchmarked). */
int hotspot_compile(const hotspot_config *cfg, char *path_out, int path_cap);

/* --------------------------------------------------------------- plain path */

/* Plans a grid: cfg, else the tuned winner of the hotspot winners cache for
 * this grid size (tuned/hotspot_winners.jsonl beside the library, or
 * $HOTSPOT_WINNERS), else the winner for another grid that is legal here
 * (4096 x 4096 first, else the most recent), else the default. Compiles and
 * loads the kernel.
 * Source: Section 5 (the hotspot benchmark kernel) with a point of the
 * Table 1 space. */
int hotspot_plan(hotspot_plan_t *plan, hotspot_shape s, const hotspot_config *cfg);

/* The plan's configuration; *tuned = 1 when it is this grid's winner, 2
 * when it is another grid's, 0 otherwise (given or default).
 * Source: Table 1 (the parameters of the configuration). */
int hotspot_plan_config(hotspot_plan_t plan, hotspot_config *cfg, int *tuned);

/* d_out = the grid after `steps` (>= 0) steps from d_temp, on `stream`:
 * ceil(steps / temporal) launches that alternate between d_out and d_work, so
 * that the last writes d_out. d_work (rows*cols floats) may be NULL when one
 * launch suffices. d_temp and d_power are read only; d_out and d_work must
 * not overlap each other or the inputs.
 * Source: Section 5 (the hotspot kernel) and Section 6.2 (temporal tiling:
 * several steps per launch, with redundant halo work); the update is the
 * thermal model stated at the top of this header. */
int hotspot_run(hotspot_plan_t plan, const float *d_temp, const float *d_power, float *d_out, float *d_work,
                int steps, hotspot_coeffs k, void *stream);

/* Cells of the fixed work grid of hotspot_run_noalloc (64 MiB of FP32). */
#define HOTSPOT_NOALLOC_CELLS (4096 * 4096)

/* hotspot_run without a work buffer and without any allocation, for callers
 * that cannot allocate device memory (code under graph capture, serving
 * loops or harnesses that forbid hipMalloc). A run of more than one launch
 * alternates between d_out and a fixed work grid of the library's own device
 * code (HOTSPOT_NOALLOC_CELLS floats on every GPU the library runs on, kept
 * until the process ends); grids of more cells need more than one launch
 * only when steps > temporal, and then return CONV2D_EINVAL. The results are
 * those of hotspot_run, bit for bit. Every call on one GPU uses that GPU's
 * one work grid: calls that overlap on a GPU (other streams or host
 * threads) race, so the caller orders them. The grid's contents are not
 * kept from call to call (every launch overwrites what it reads later).
 * Source: none in the paper (the variant of hotspot_run for callers that
 * cannot allocate). */
int hotspot_run_noalloc(hotspot_plan_t plan, const float *d_temp, const float *d_power, float *d_out, int steps,
                        hotspot_coeffs k, void *stream);

/* Frees the plan and unloads its code objects. It does not wait:
 * the caller first makes sure that no launch of the plan is queued or
 * running (synchronize the streams it ran on) and that no graph holding its
 * kernels is replayed afterwards. NULL is ignored.
 * Source: none in the paper (resource release of this ABI). */
void hotspot_destroy(hotspot_plan_t plan);

/* The same computation one step per launch, one cell per thread (the tuner's
 * bitwise reference). Buffers as for hotspot_run.
 * Source: Section 5 (the hotspot kernel's result without temporal tiling). */
int hotspot_reference(hotspot_shape s, const float *d_temp, const float *d_power, float *d_out, float *d_work,
                      int steps, hotspot_coeffs k, void *stream);

/* --------------------------------------------------------------- tuner */

typedef struct hotspot_tune_opts {
    const char *winners_path;  /* winners cache to append to (NULL: do not cache) */
    const char *results_path;  /* per-configuration results (JSON lines; resumable), or NULL */
    int warmup;                /* untimed runs per point (default 2) */
    int reps;                  /* timed runs per point, median taken (default 20) */
    int retime_reps;           /* sustained runs re-timing the ten fastest (default 200) */
    int flush_mall;            /* 1: read 512 MiB between timed runs (default 1) */
    int threads;               /* compile threads (0: hardware threads, at most 16) */
    int max_configs;           /* first N legal points only (0: all) */
    double tie_rel;            /* times within this fraction of the fastest tie (default 0.005) */
    int verbose;
} hotspot_tune_opts;

typedef struct hotspot_tune_result {
    hotspot_config best;
    double best_ms, default_ms, median_ms;       /* one hotspot_run of `steps` steps; best_ms and
                                                    default_ms in the re-timing's sustained mode
                                                    (the sweep's when retime_reps = 0) */
    double best_gflops, median_gflops, default_gflops;
    double impact;                               /* best over median throughput (Section 4) */
    int n_space, n_illegal, n_compile_fail, n_launch_fail, n_verify_fail, n_timed, n_resumed;
    int default_rank;                            /* 1 = fastest; 0 if the default was not timed */
    hotspot_config top[5];
    double top_ms[5];
    double compile_s, measure_s;
    double best_sweep_ms, default_sweep_ms;      /* the sweep's flushed times (0 if not timed) */
} hotspot_tune_result;

/* Source: none in the paper (option defaults). */
void hotspot_tune_defaults(hotspot_tune_opts *o);

/* Sweeps the restricted space for grid s and `steps` steps per run (each
 * point compiled, verified bitwise against hotspot_reference on seeded data,
 * timed as a whole hotspot_run after a cache flush, median of `reps`),
 * re-times the ten fastest with sustained runs (as conv2d_tune), picks the
 * winner (lowest sustained time; ties within tie_rel to the smallest tuple)
 * and appends it to the winners cache. Throughput counts 14 floating-point
 * operations per cell and step.
 * Source: Section 3 (compile, then time each configuration with events);
 * Section 4 (tuning impact, as in Table 3); Table 1 (the space); Table 5
 * (the top configurations this reproduces on MI355X). */
int hotspot_tune(hotspot_shape s, int steps, const hotspot_tune_opts *opts, hotspot_tune_result *res);

#ifdef __cplusplus
}
#endif

#endif /* HOTSPOT_H */
