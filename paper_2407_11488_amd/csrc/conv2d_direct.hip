// Direct 2D image convolution for gfx950 (CDNA4), one tunable configuration
// per compilation. The host library compiles this file at run time with
// hiprtc, once per (configuration, filter size, alignment class), the way the
// paper's tuner compiles each point of its search space (Section 3; the
// convolution's tunable parameters are Table 1).
//
// Computes, for 0 <= y < H, 0 <= x < W (valid cross-correlation, no flip):
//     out[y][x] = sum_{i<FH} sum_{j<FW} in[y+i][x+j] * f[i][j]
// with `in` (H+FH-1) x (W+FW-1), `f` FH x FW, `out` H x W, row-major FP32.
//
// Accumulation order is fixed for every configuration: one FP32 accumulator
// per output, fused multiply-add, taps in i-ascending then j-ascending order.
// Every configuration (and the batched kernel) therefore returns the same
// bits for the same inputs.
//
// Compile-time parameters (-D):
//   CONV_BX, CONV_BY   workgroup shape in threads (block_size_x / block_size_y)
//   CONV_TX, CONV_TY   outputs per thread along x and y (tile_size_x / _y)
//   CONV_USE_LDS       1: the workgroup stages its input halo tile in LDS
//   CONV_FCONST        1: filter copied into this module's __constant__ array
//                      0: filter read through a const __restrict__ pointer
//   CONV_UNROLL        unroll of the input-row loop (0 = full)
//   CONV_FH, CONV_FW   filter size
//   CONV_VIN           input vector width 1/2/4
//   CONV_VOUT          output vector width 1/2/4
//                      The library builds every kernel with 4 and 4, for rows
//                      of any width: a gfx9-family access of several dwords
//                      needs only dword alignment in the alignment mode the
//                      ROCm driver sets, and a raw buffer load checks each
//                      dword against the buffer size (a vector that straddles
//                      the end of the input reads zeros past it).
//   CONV_NAME          kernel symbol (one per configuration, so that profiles
//                      tell configurations apart); default conv2d_direct
//   CONV_BATCH         1: build the batched kernel (many images of
//                      one filter size, described in device memory) instead
//
// Design (MI355X):
//  * Each thread owns a TY x TX register tile of outputs, contiguous in x.
//    It walks the TY+FH-1 input rows its tile needs once each: a row window of
//    TX+FW-1 values is loaded into VGPRs and feeds every output row that uses
//    it (TY*TX*FW FMAs per window in the steady state). Filter taps are wave
//    uniform and are read with scalar loads, so each FMA is
//    v_fmac_f32 acc, s_tap, v_in.
//  * Global reads use raw buffer loads: an out-of-range dword reads 0
//    instead of faulting, so edge tiles need no clamping; outputs outside the
//    image are simply not stored.
//  * Workgroup ids are remapped so that each of the 8 XCDs (dispatched
//    round-robin) receives one contiguous run of tiles, keeping vertically
//    adjacent tiles, which share FH-1 input rows, in the same L2.

#ifndef CONV_BATCH
#define CONV_BATCH 0
#endif

#ifndef CONV_BX
#error "CONV_BX must be defined"
#endif

#ifndef CONV_NAME
#define CONV_NAME conv2d_direct
#endif

typedef unsigned int u32;
typedef u32 u32x2 __attribute__((ext_vector_type(2)));
typedef u32 u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

static constexpr int gcd4(int t) { return (t % 4 == 0) ? 4 : ((t % 2 == 0) ? 2 : 1); }
static constexpr int min_(int a, int b) { return a < b ? a : b; }

// Derived sizes of one configuration (filter FH x FW, workgroup BX x BY
// threads, TX x TY outputs per thread, LDS staging on/off, row-loop unroll,
// input/output vector widths).
template <int FH, int FW, int BX, int BY, int TX, int TY, int LDS, int UNROLL, int VIN, int VOUT>
struct Geo {
    static constexpr int NT = BX * BY;
    static constexpr int WIN = TX + FW - 1;      // input values a thread's row window needs
    static constexpr int NROWS = TY + FH - 1;    // input rows a thread walks
    // Vector width of a thread's window loads: min(gcd(TX, 4), VIN) from
    // global memory, gcd(TX, 4) from LDS (pitch a multiple of 4, the window
    // starting at a multiple of TX, so LDS reads stay aligned). The register
    // window is padded to a whole number of those vectors.
    static constexpr int WVEC = LDS ? gcd4(TX) : min_(gcd4(TX), VIN);
    static constexpr int WIN_PAD = ((WIN + WVEC - 1) / WVEC) * WVEC;
    static constexpr int SVEC = min_(gcd4(TX), VOUT);   // output store width
    // Input halo tile of one workgroup in LDS, rows x pitch floats. The pitch
    // is padded to a multiple of 4 (aligned ds_read_b128) plus 4 when it would
    // otherwise be a multiple of 32 banks' worth, to spread the rows a wave
    // reads over banks.
    static constexpr int LDS_ROWS = BY * TY + FH - 1;
    static constexpr int LDS_COLS = BX * TX + FW - 1;
    static constexpr int LDS_CHUNKS = (LDS_COLS + VIN - 1) / VIN;
    static constexpr int LDS_PITCH0 = ((LDS_CHUNKS * VIN + 3) / 4) * 4;
    static constexpr int LDS_PITCH = (LDS_PITCH0 % 32 == 0) ? LDS_PITCH0 + 4 : LDS_PITCH0;
    static constexpr int LDS_FLOATS = LDS ? LDS_ROWS * LDS_PITCH : 4;
    static constexpr int ROW_UNROLL = UNROLL == 0 ? NROWS : UNROLL;   // 0 = the whole row loop
};

// Filter taps: the module's __constant__ copy, or the filter pointer.
#if CONV_FCONST
__constant__ float conv_filter[CONV_FH * CONV_FW];
#define TAPS conv_filter
#else
#define TAPS filt
#endif

static __device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const float* p, u32 bytes)
{
    // Word 3 = 0x00020000: raw (untyped) dword access, the gfx9-family value.
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, 0x00020000);
}

// Loads N consecutive floats from byte offset `off` of the buffer into dst[0..N).
// Whole vectors are bit-cast: bit-casting a single ext-vector element
// (v.y, ...) is miscompiled by this clang into a read of element 0.
template <int V, int N>
static __device__ __forceinline__ void buffer_row(float* dst, __amdgpu_buffer_rsrc_t rs, u32 off)
{
#pragma unroll
    for (int m = 0; m < N; m += V) {
        if constexpr (V == 4) {
            f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(off + 4u * m), 0, 0));
            dst[m + 0] = v.x;
            dst[m + 1] = v.y;
            dst[m + 2] = v.z;
            dst[m + 3] = v.w;
        } else if constexpr (V == 2) {
            f32x2 v = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(off + 4u * m), 0, 0));
            dst[m + 0] = v.x;
            dst[m + 1] = v.y;
        } else {
            u32 v = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(off + 4u * m), 0, 0);
            dst[m] = __builtin_bit_cast(float, v);
        }
    }
}

// Loads N consecutive floats from LDS (V-element aligned) into dst[0..N).
template <int V, int N>
static __device__ __forceinline__ void lds_row(float* dst, const float* src)
{
#pragma unroll
    for (int m = 0; m < N; m += V) {
        if constexpr (V == 4) {
            f32x4 v = *(const f32x4*)(src + m);
            dst[m + 0] = v.x; dst[m + 1] = v.y; dst[m + 2] = v.z; dst[m + 3] = v.w;
        } else if constexpr (V == 2) {
            f32x2 v = *(const f32x2*)(src + m);
            dst[m + 0] = v.x; dst[m + 1] = v.y;
        } else {
            dst[m] = src[m];
        }
    }
}

// Workgroup id -> tile id: XCD x (= id mod 8) gets the contiguous tile range
// [start(x), start(x) + count(x)); a bijection on [0, n_tiles).
static __device__ __forceinline__ int xcd_remap(int id, int n_tiles)
{
    const int q = n_tiles >> 3, rem = n_tiles & 7;
    const int xcd = id & 7, k = id >> 3;
    return xcd * q + min_(xcd, rem) + k;
}

// One output tile of (BY*TY) x (BX*TX) at tile coordinates (tile_y, tile_x)
// of an image. Every thread of the workgroup calls it (the LDS variant
// contains a barrier). `lds` is the workgroup's LDS tile.
template <int FH, int FW, int BX, int BY, int TX, int TY, int LDS, int UNROLL, int VIN, int VOUT>
static __device__ __forceinline__ void conv_tile(const float* __restrict__ in, const float* __restrict__ filt,
                                                 float* __restrict__ out, int H, int W, u32 in_bytes,
                                                 int tile_x, int tile_y, float* __restrict__ lds)
{
    using G = Geo<FH, FW, BX, BY, TX, TY, LDS, UNROLL, VIN, VOUT>;
    const int lx = (int)threadIdx.x % BX;
    const int ly = (int)threadIdx.x / BX;
    const int x0 = tile_x * (BX * TX) + lx * TX;
    const int y0 = tile_y * (BY * TY) + ly * TY;
    const u32 P = (u32)W + (FW - 1);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(in, in_bytes);

    const float* lbase = lds;
    if constexpr (LDS) {
        const u32 gx0 = (u32)tile_x * (BX * TX);
        const u32 gy0 = (u32)tile_y * (BY * TY);
        for (int c = (int)threadIdx.x; c < G::LDS_ROWS * G::LDS_CHUNKS; c += G::NT) {
            const int rr = c / G::LDS_CHUNKS;
            const int cc = (c - rr * G::LDS_CHUNKS) * VIN;
            float v[VIN];
            buffer_row<VIN, VIN>(v, rs, ((gy0 + rr) * P + gx0 + cc) * 4u);
#pragma unroll
            for (int m = 0; m < VIN; ++m)
                lds[rr * G::LDS_PITCH + cc + m] = v[m];
        }
        __syncthreads();
        lbase = lds + (ly * TY) * G::LDS_PITCH + lx * TX;
    }

    if (x0 >= W || y0 >= H)
        return;

    float acc[TY][TX];
#pragma unroll
    for (int o = 0; o < TY; ++o)
#pragma unroll
        for (int k = 0; k < TX; ++k)
            acc[o][k] = 0.0f;

    const u32 off0 = ((u32)y0 * P + (u32)x0) * 4u;

#pragma unroll G::ROW_UNROLL
    for (int r = 0; r < G::NROWS; ++r) {
        float w[G::WIN_PAD];
        if constexpr (LDS)
            lds_row<G::WVEC, G::WIN_PAD>(w, lbase + r * G::LDS_PITCH);
        else
            buffer_row<G::WVEC, G::WIN_PAD>(w, rs, off0 + (u32)r * P * 4u);
#pragma unroll
        for (int o = 0; o < TY; ++o) {
            const int i = r - o;
            if (i >= 0 && i < FH) {
#pragma unroll
                for (int j = 0; j < FW; ++j) {
                    const float fv = TAPS[i * FW + j];
#pragma unroll
                    for (int k = 0; k < TX; ++k)
                        acc[o][k] = __builtin_fmaf(w[k + j], fv, acc[o][k]);
                }
            }
        }
    }

#pragma unroll
    for (int o = 0; o < TY; ++o) {
        const int y = y0 + o;
        if (y < H) {
            float* orow = out + (size_t)y * (size_t)W + x0;
            if (x0 + TX <= W) {
#pragma unroll
                for (int k = 0; k < TX; k += G::SVEC) {
                    if constexpr (G::SVEC == 4) {
                        f32x4 v = {acc[o][k], acc[o][k + 1], acc[o][k + 2], acc[o][k + 3]};
                        __builtin_nontemporal_store(v, (f32x4*)(orow + k));
                    } else if constexpr (G::SVEC == 2) {
                        f32x2 v = {acc[o][k], acc[o][k + 1]};
                        __builtin_nontemporal_store(v, (f32x2*)(orow + k));
                    } else {
                        __builtin_nontemporal_store(acc[o][k], orow + k);
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < TX; ++k)
                    if (x0 + k < W)
                        orow[k] = acc[o][k];
            }
        }
    }
}

#if CONV_BATCH == 0
// One image: one workgroup per tile, tiles_x * tiles_y = n_tiles workgroups.
using G1 = Geo<CONV_FH, CONV_FW, CONV_BX, CONV_BY, CONV_TX, CONV_TY, CONV_USE_LDS, CONV_UNROLL, CONV_VIN, CONV_VOUT>;
extern "C" __global__ void __launch_bounds__(G1::NT)
CONV_NAME(const float* __restrict__ in, const float* __restrict__ filt,
          float* __restrict__ out, int H, int W, int tiles_x, int n_tiles, u32 in_bytes)
{
    __shared__ __attribute__((aligned(16))) float lds[G1::LDS_FLOATS];
    const int t = xcd_remap((int)blockIdx.x, n_tiles);
    const int tile_y = t / tiles_x;
    const int tile_x = t - tile_y * tiles_x;
    conv_tile<CONV_FH, CONV_FW, CONV_BX, CONV_BY, CONV_TX, CONV_TY, CONV_USE_LDS, CONV_UNROLL, CONV_VIN, CONV_VOUT>(
        in, filt, out, H, W, in_bytes, tile_x, tile_y, lds);
}
#else
#if CONV_FCONST
#error "the batched kernel reads each problem's own filter through its pointer"
#endif
// One problem of a batch, as the host library lays it out in device memory.
struct ConvDesc {
    const float* in;
    const float* filt;
    float* out;
    int H, W;
    int tiles_x;
    int tile_begin;   // first tile of this problem in the tile list
    u32 in_bytes;
    int n_tiles;      // tiles of this problem
};

// The descriptor of tile t. The owner is read with a 16-bit vector load (no
// 16-bit scalar load on gfx9); it is the same for every lane, and saying so
// keeps the descriptor, the filter taps and all addressing in scalar registers.
static __device__ __forceinline__ const ConvDesc* tile_desc(const ConvDesc* __restrict__ descs,
                                                            const unsigned short* __restrict__ owner, int t)
{
    return descs + __builtin_amdgcn_readfirstlane((int)owner[t]);
}

// Many images with the same filter size: a grid of at least 8 workgroups
// walks the group's tile list (the library launches one workgroup per tile;
// a smaller grid gives each workgroup several). The tiles of XCD x (=
// workgroup id mod 8) form one contiguous range, shared out by stride among
// that XCD's workgroups; owner[t] names the problem of tile t.
using G1 = Geo<CONV_FH, CONV_FW, CONV_BX, CONV_BY, CONV_TX, CONV_TY, CONV_USE_LDS, CONV_UNROLL, CONV_VIN, CONV_VOUT>;
extern "C" __global__ void __launch_bounds__(G1::NT)
CONV_NAME(const ConvDesc* __restrict__ descs, const unsigned short* __restrict__ owner, int total_tiles)
{
    __shared__ __attribute__((aligned(16))) float lds[G1::LDS_FLOATS];
    const int G = (int)gridDim.x;
    const int xcd = (int)blockIdx.x & 7;
    const int first = (int)blockIdx.x >> 3;
    const int stride = (G - xcd + 7) >> 3;
    const int q = total_tiles >> 3, rem = total_tiles & 7;
    const int begin = xcd * q + min_(xcd, rem);
    const int count = q + (xcd < rem ? 1 : 0);
    for (int k = first; k < count; k += stride) {
        const int t = begin + k;
        const ConvDesc* d = tile_desc(descs, owner, t);
        const int lt = t - d->tile_begin;
        if ((unsigned)lt >= (unsigned)d->n_tiles)
            continue;  // inconsistent tables: skip rather than store out of range (uniform)
        const int tile_y = lt / d->tiles_x;
        const int tile_x = lt - tile_y * d->tiles_x;
        if (CONV_USE_LDS && k != first)
            __syncthreads();  // every thread is done with the previous tile's LDS
        conv_tile<CONV_FH, CONV_FW, CONV_BX, CONV_BY, CONV_TX, CONV_TY, CONV_USE_LDS, CONV_UNROLL, CONV_VIN, CONV_VOUT>(
            d->in, d->filt, d->out, d->H, d->W, d->in_bytes, tile_x, tile_y, lds);
    }
}
#endif
