// Hotspot thermal stencil for gfx950 (CDNA4) with temporal tiling, one
// tunable configuration per compilation (the paper's hotspot kernel and its
// tunable parameters, Section 5 and Table 1; the computation is the compact
// thermal RC model of a chip, Huang et al., HotSpot, IEEE TVLSI 2006).
//
// One explicit step on a rows x cols grid of temperatures T and powers P:
//   T'[r][c] = T + cc * (P + (T[r-1][c] + T[r+1][c] - 2T) * gy
//                          + (T[r][c-1] + T[r][c+1] - 2T) * gx
//                          + (t_amb - T) * gz)
// where a neighbour outside the grid is the cell itself. The kernel evaluates
// the same step with its terms grouped by what they multiply,
//   T' = a*T + ky*(N + S) + kx*(W + E) + s,   s = cc*P + q,
// a = 1 - cc*(2gx + 2gy + gz), ky = cc*gy, kx = cc*gx, q = cc*gz*t_amb
// (folded by the host): two neighbour sums and three fused multiply-adds per
// cell and step, s once per cell and launch when power stays on chip. Every
// cell is evaluated in the same order, so every configuration returns the
// same bits.
//
// Compile-time parameters (-D):
//   HS_BX, HS_BY   workgroup shape in threads (block_size_x / block_size_y)
//   HS_TX, HS_TY   cells per thread along x and y (tile_size_x / _y)
//   HS_TT          temporal tiling factor: steps per launch (at most)
//   HS_UNROLL_T    1: rolled step loop; 0: fully unrolled (loop_unroll_factor_t)
//   HS_SH_POWER    1: each thread keeps its cells' power on chip for all steps;
//                  0: power is read from global memory at every step (sh_power)
//   HS_NAME        kernel symbol
//
// Design (MI355X): a workgroup owns a region of (BY*TY) x (BX*TX) cells, its
// output tile plus a halo of TT cells on every side; neighbouring regions
// overlap by 2*TT. Each thread keeps its TY x TX cells in VGPRs through all
// steps, and per step exchanges its edge cells with the neighbouring threads
// through one of two LDS buffers (used alternately, so one barrier per step):
//  * BX <= 64 (a wave holds whole thread rows): horizontal neighbours come
//    straight from the adjacent lanes (DPP wave shifts, folded into the
//    adds); only each thread row's top and bottom cell rows go through LDS.
//  * BX > 64: every cell is published to a copy of the region in LDS (with
//    a zero ring) and the threads read the ring of cells around their tile.
// A lane at the end of a thread row gets its outside neighbour from the next
// thread row, or zero: such cells lie on the region's edge, whose values are
// not exact anyway.
// After s steps the cells at distance >= s from the region's edge are exact;
// after the launch's steps (<= TT) the inner tile is stored. The grid edge is
// handled by coordinates, never by reading outside the grid. A region inside
// the grid reads and writes through raw buffers based at its first cell
// (32-bit offsets: one address per thread, rows by a scalar offset), with
// every load issued before the first one is waited for.

#ifndef HS_BX
#error "HS_BX must be defined"
#endif
#ifndef HS_NAME
#define HS_NAME hotspot_step
#endif

#define HS_NT (HS_BX * HS_BY)
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

#define RH (HS_BY * HS_TY)   // region rows
#define RW (HS_BX * HS_TX)   // region columns
#define OH (RH - 2 * HS_TT)  // output tile rows
#define OW (RW - 2 * HS_TT)  // output tile columns
// LDS buffer: the region plus a one-cell ring (cell (R, C) at LIDX(R, C)),
// so that every neighbour read of a region cell stays inside the buffer and
// needs no test; ring cells are zero and feed only cells that are not exact
// anyway. Odd pitch: a wave's column reads spread over the banks.
#define LDS_PITCH ((RW + 2) | 1)
#define LDS_CELLS ((RH + 2) * LDS_PITCH)
#define LIDX(R, C) (((R) + 1) * LDS_PITCH + (C) + 1)
// Row exchange (BX <= 64): for thread row ly, its top cell row at
// XIDX(2 * ly + 2, C) and its bottom row at XIDX(2 * ly + 3, C); rows 1
// (above thread row 0) and 2 * BY + 2 (below the last) stay zero.
#define HS_ROWX (HS_BX <= 64)
#define XROWS (2 * HS_BY + 4)
#define XIDX(Q, C) ((Q) * RW + (C))
#if HS_ROWX
#define HS_LDS_FLOATS (XROWS * RW)
#if 64 % HS_BX != 0
#error "block_x must divide the wave size"
#endif
#else
#define HS_LDS_FLOATS LDS_CELLS
#endif

#if OH < 1 || OW < 1
#error "the region must be larger than twice the temporal tiling factor"
#endif

static __device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// A raw buffer over `bytes` bytes from p (dword access; word 3 is the gfx9
// family's raw-buffer value).
static __device__ __forceinline__ __amdgpu_buffer_rsrc_t region_rsrc(const float* p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, 0x00020000);
}

// Workgroup id -> tile id: XCD x (= id mod 8) gets one contiguous run of
// tiles, so neighbouring tiles, which share halo cells, meet in one L2.
static __device__ __forceinline__ int xcd_remap(int id, int n_tiles)
{
    const int q = n_tiles >> 3, rem = n_tiles & 7;
    const int xcd = id & 7, k = id >> 3;
    return xcd * q + (xcd < rem ? xcd : rem) + k;
}

// The value of x in the lane below (lane i - 1; lane 0 gets 0) and above
// (lane i + 1; lane 63 gets 0): DPP wave shifts.
static __device__ __forceinline__ float lane_below(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138, 0xf, 0xf, true));
}
static __device__ __forceinline__ float lane_above(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xf, 0xf, true));
}

// A cell's source term: its power and the ambient's share, per step.
static __device__ __forceinline__ float source(float p, float cc, float q) { return __builtin_fmaf(cc, p, q); }

static __device__ __forceinline__ float cell_step(float t, float north, float south, float west, float east, float src,
                                                  float ka, float ky, float kx)
{
    float x = __builtin_fmaf(kx, west + east, src);
    x = __builtin_fmaf(ky, north + south, x);
    return __builtin_fmaf(ka, t, x);
}

// The launch's steps over the thread's cells v (in place). EDGE = false when
// the workgroup's whole region lies inside the grid: no cell then needs the
// grid-edge rule, and the per-cell coordinate tests disappear.
template <bool EDGE>
static __device__ __forceinline__ void run_steps(float (&v)[HS_TY][HS_TX], const float (&pw)[HS_TY][HS_TX],
                                                 float (*buf)[HS_LDS_FLOATS], const float* __restrict__ power,
                                                 int rows, int cols, int steps, int R0, int C0, int gr0, int gc0,
                                                 float ka, float ky, float kx, float cc, float q)
{
    const int ly = R0 / HS_TY;
#if HS_UNROLL_T
#pragma unroll 1
#else
#pragma unroll
#endif
    for (int s = 0; s < HS_TT; ++s) {
        if (s >= steps)
            break;
        float* cur = buf[s & 1];
#if HS_ROWX
#pragma unroll
        for (int b = 0; b < HS_TX; ++b) {
            cur[XIDX(2 * ly + 2, C0 + b)] = v[0][b];
            cur[XIDX(2 * ly + 3, C0 + b)] = v[HS_TY - 1][b];
        }
#else
#pragma unroll
        for (int a = 0; a < HS_TY; ++a)
#pragma unroll
            for (int b = 0; b < HS_TX; ++b)
                cur[LIDX(R0 + a, C0 + b)] = v[a][b];
#endif
        __syncthreads();

        float nv[HS_TY][HS_TX];
#pragma unroll
        for (int a = 0; a < HS_TY; ++a) {
            const int R = R0 + a, gr = gr0 + a;
#if HS_ROWX
            // every lane takes part in the shifts, whatever its cells need
            const float from_west = lane_below(v[a][HS_TX - 1]);
            const float from_east = lane_above(v[a][0]);
#endif
#pragma unroll
            for (int b = 0; b < HS_TX; ++b) {
                const int C = C0 + b, gc = gc0 + b;
                const float t = v[a][b];
                // Neighbours: the cell itself at the grid's edge; a register
                // inside the thread's block; else another thread's cell (at
                // the region's own edge, zero: such cells are never exact).
                float north, south, west, east;
#if HS_ROWX
                (void)R;
                (void)C;
                north = a > 0 ? v[a - 1][b] : cur[XIDX(2 * ly + 1, C0 + b)];
                south = a < HS_TY - 1 ? v[a + 1][b] : cur[XIDX(2 * ly + 4, C0 + b)];
                west = b > 0 ? v[a][b - 1] : from_west;
                east = b < HS_TX - 1 ? v[a][b + 1] : from_east;
                if (EDGE) {
                    north = gr == 0 ? t : north;
                    south = gr == rows - 1 ? t : south;
                    west = gc == 0 ? t : west;
                    east = gc == cols - 1 ? t : east;
                }
#else
                if (EDGE && gr == 0) north = t;
                else if (a > 0) north = v[a - 1][b];
                else north = cur[LIDX(R - 1, C)];
                if (EDGE && gr == rows - 1) south = t;
                else if (a < HS_TY - 1) south = v[a + 1][b];
                else south = cur[LIDX(R + 1, C)];
                if (EDGE && gc == 0) west = t;
                else if (b > 0) west = v[a][b - 1];
                else west = cur[LIDX(R, C - 1)];
                if (EDGE && gc == cols - 1) east = t;
                else if (b < HS_TX - 1) east = v[a][b + 1];
                else east = cur[LIDX(R, C + 1)];
#endif
#if HS_SH_POWER
                const float src = pw[a][b];
                (void)cc;
                (void)q;
#else
                const float src =
                    source(power[(size_t)clampi(gr, 0, rows - 1) * (size_t)cols + clampi(gc, 0, cols - 1)], cc, q);
#endif
                nv[a][b] = cell_step(t, north, south, west, east, src, ka, ky, kx);
            }
        }
#pragma unroll
        for (int a = 0; a < HS_TY; ++a)
#pragma unroll
            for (int b = 0; b < HS_TX; ++b)
                v[a][b] = nv[a][b];
    }
}

extern "C" __global__ void __launch_bounds__(HS_NT)
HS_NAME(const float* __restrict__ tin, const float* __restrict__ power, float* __restrict__ tout, int rows,
        int cols, int steps, int tiles_x, int n_tiles, float ka, float ky, float kx, float cc, float q)
{
    __shared__ __attribute__((aligned(16))) float buf[2][HS_LDS_FLOATS];
    const int tile = xcd_remap((int)blockIdx.x, n_tiles);
    const int tile_y = tile / tiles_x;
    const int tile_x = tile - tile_y * tiles_x;
    const int lx = (int)threadIdx.x % HS_BX;
    const int ly = (int)threadIdx.x / HS_BX;
    const int R0 = ly * HS_TY, C0 = lx * HS_TX;           // first cell of this thread in the region
    const int rr0 = tile_y * OH - HS_TT, rc0 = tile_x * OW - HS_TT;   // the region's first global cell
    const int gr0 = rr0 + R0, gc0 = rc0 + C0;              // the thread's first global cell

    // Workgroup-uniform: does the region touch (or cross) the grid's edge?
    // (Regions whose rows span 2^31 bytes or more take the same clamped path.)
    const bool edge = rr0 <= 0 || rc0 <= 0 || rr0 + RH >= rows || rc0 + RW >= cols ||
                      (long long)RH * (long long)cols >= (1ll << 29);
    // Inside the grid, the region's rows are one buffer starting at its first
    // cell; a thread's cell (a, b) sits at byte voff + 4 * (a * cols + b).
    const long long rbase = (long long)rr0 * (long long)cols + (long long)rc0;
    const unsigned rbytes = (unsigned)(RH * cols) * 4u;
    const unsigned voff = (unsigned)(R0 * cols + C0) * 4u;

    // The thread's cells (and with power on chip, their source terms). At
    // the grid's edge, reads are clamped into the grid: cells outside it are
    // never stored and never feed a cell inside.
    float v[HS_TY][HS_TX];
    float pw[HS_TY][HS_TX];
    if (edge) {
#pragma unroll
        for (int a = 0; a < HS_TY; ++a) {
            const size_t row = (size_t)clampi(gr0 + a, 0, rows - 1) * (size_t)cols;
#pragma unroll
            for (int b = 0; b < HS_TX; ++b) {
                const int c = clampi(gc0 + b, 0, cols - 1);
                v[a][b] = tin[row + c];
                pw[a][b] = HS_SH_POWER ? source(power[row + c], cc, q) : 0.0f;
            }
        }
    } else {
        const __amdgpu_buffer_rsrc_t rt = region_rsrc(tin + rbase, rbytes);
        const __amdgpu_buffer_rsrc_t rp = region_rsrc(power + rbase, rbytes);
        float praw[HS_TY][HS_TX];
#pragma unroll
        for (int a = 0; a < HS_TY; ++a)
#pragma unroll
            for (int b = 0; b < HS_TX; ++b) {
                const int so = a * cols * 4;   // wave-uniform
                v[a][b] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rt, (int)(voff + 4u * b), so, 0));
                praw[a][b] = HS_SH_POWER
                    ? __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rp, (int)(voff + 4u * b), so, 0))
                    : 0.0f;
            }
        // every load is in flight before the first source term waits for one
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int a = 0; a < HS_TY; ++a)
#pragma unroll
            for (int b = 0; b < HS_TX; ++b)
                pw[a][b] = HS_SH_POWER ? source(praw[a][b], cc, q) : 0.0f;
    }

    // Zero what no thread writes (the rows around the thread rows, or the
    // region's ring) in both buffers. The first step's barrier orders these
    // writes before any read.
#if HS_ROWX
    for (int k = (int)threadIdx.x; k < 2 * RW; k += HS_NT) {
        const int q = k < RW ? 1 : 2 * HS_BY + 2, c = k < RW ? k : k - RW;
        buf[0][XIDX(q, c)] = 0.0f;
        buf[1][XIDX(q, c)] = 0.0f;
    }
#else
    for (int k = (int)threadIdx.x; k < 2 * (RW + 2) + 2 * RH; k += HS_NT) {
        int r, c;
        if (k < RW + 2) { r = -1; c = k - 1; }
        else if (k < 2 * (RW + 2)) { r = RH; c = k - (RW + 2) - 1; }
        else { r = (k - 2 * (RW + 2)) >> 1; c = (k & 1) ? RW : -1; }
        buf[0][LIDX(r, c)] = 0.0f;
        buf[1][LIDX(r, c)] = 0.0f;
    }
#endif

    if (edge)
        run_steps<true>(v, pw, buf, power, rows, cols, steps, R0, C0, gr0, gc0, ka, ky, kx, cc, q);
    else
        run_steps<false>(v, pw, buf, power, rows, cols, steps, R0, C0, gr0, gc0, ka, ky, kx, cc, q);

    // Store the inner tile (cells at least TT from the region's edge; at the
    // grid's edge, those inside the grid).
    if (edge) {
        const long long base = (long long)gr0 * (long long)cols + (long long)gc0;
#pragma unroll
        for (int a = 0; a < HS_TY; ++a) {
            const int R = R0 + a, gr = gr0 + a;
            if (R < HS_TT || R >= RH - HS_TT || gr >= rows)
                continue;
            const long long row = base + (long long)a * (long long)cols;
#pragma unroll
            for (int b = 0; b < HS_TX; ++b) {
                const int C = C0 + b, gc = gc0 + b;
                if (C >= HS_TT && C < RW - HS_TT && gc < cols)
                    tout[row + b] = v[a][b];
            }
        }
    } else {
        const __amdgpu_buffer_rsrc_t ro = region_rsrc(tout + rbase, rbytes);
#pragma unroll
        for (int a = 0; a < HS_TY; ++a) {
            const int R = R0 + a;
            if (R < HS_TT || R >= RH - HS_TT)
                continue;
            if constexpr (HS_TX % 2 == 0) {
                // Two neighbouring outputs of the output tile go out as one
                // two-dword store (it needs only dword alignment): half the
                // store instructions, each writing whole 8-byte pairs.
#pragma unroll
                for (int b = 0; b < HS_TX; b += 2) {
                    const int C = C0 + b;
                    const bool in0 = C >= HS_TT && C < RW - HS_TT;
                    const bool in1 = C + 1 >= HS_TT && C + 1 < RW - HS_TT;
                    if (in0 && in1) {
                        const u32x2 w = {__builtin_bit_cast(unsigned, v[a][b]),
                                         __builtin_bit_cast(unsigned, v[a][b + 1])};
                        __builtin_amdgcn_raw_buffer_store_b64(w, ro, (int)(voff + 4u * b), a * cols * 4, 0);
                    } else {
                        if (in0)
                            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v[a][b]), ro,
                                                                  (int)(voff + 4u * b), a * cols * 4, 0);
                        if (in1)
                            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v[a][b + 1]), ro,
                                                                  (int)(voff + 4u * (b + 1)), a * cols * 4, 0);
                    }
                }
            } else {
#pragma unroll
                for (int b = 0; b < HS_TX; ++b) {
                    const int C = C0 + b;
                    if (C >= HS_TT && C < RW - HS_TT)
                        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v[a][b]), ro,
                                                              (int)(voff + 4u * b), a * cols * 4, 0);
                }
            }
        }
    }
}
