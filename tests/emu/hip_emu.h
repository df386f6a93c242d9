// Host emulation of the HIP device features the convolution kernels use, so
// the kernel sources compile as ordinary C++ and run on the CPU under
// AddressSanitizer: every GPU thread of a workgroup is a host thread, and
// __syncthreads() is a real barrier. Raw buffer loads keep their hardware
// meaning (an offset at or past num_records reads 0) and additionally check
// that every in-range read lies inside the allocation the buffer describes.
// Test infrastructure only.
#pragma once

#include <barrier>
#include <cassert>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __constant__
#define __shared__ static

struct emu_dim3 {
    unsigned x = 0, y = 0, z = 0;
};
extern thread_local emu_dim3 threadIdx;
extern thread_local emu_dim3 blockIdx;
extern emu_dim3 blockDim;
extern emu_dim3 gridDim;
extern std::barrier<>* emu_block_barrier;

inline void __syncthreads() { emu_block_barrier->arrive_and_wait(); }

// DPP wave shifts by one lane (wave_shr:1 = 0x138: lane i reads lane i-1;
// wave_shl:1 = 0x130: lane i reads lane i+1), 64-lane waves, lanes outside
// the wave reading 0 (bound_ctrl) or `old`. Every thread of a wave must
// call it together (as the kernels do: the shifts sit in wave-uniform
// control flow): each publishes its value, waits for its wave, reads its
// neighbour's, waits again.
extern int* emu_dpp_slots;                  // blockDim.x ints, set by the launcher
extern std::barrier<>** emu_wave_barriers;  // one per 64-lane wave of the block, set by the launcher
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl)
{
    assert(row_mask == 0xf && bank_mask == 0xf && (ctrl == 0x138 || ctrl == 0x130));
    const unsigned t = threadIdx.x, lane = t % 64, wave0 = t - lane;
    std::barrier<>* wave = emu_wave_barriers[t / 64];
    emu_dpp_slots[t] = src;
    wave->arrive_and_wait();
    int r;
    if (ctrl == 0x138)
        r = lane == 0 ? (bound_ctrl ? 0 : old) : emu_dpp_slots[wave0 + lane - 1];
    else
        r = lane == 63 ? (bound_ctrl ? 0 : old) : emu_dpp_slots[wave0 + lane + 1];
    wave->arrive_and_wait();
    return r;
}

struct __amdgpu_buffer_rsrc_t {
    const char* base;
    uint32_t num_records;
};

inline __amdgpu_buffer_rsrc_t __builtin_amdgcn_make_buffer_rsrc(void* p, short stride, int num, int flags)
{
    assert(stride == 0 && flags == 0x00020000);
    return {static_cast<const char*>(p), static_cast<uint32_t>(num)};
}

// Bytes [off, off+n) of the buffer; each dword outside num_records reads 0.
inline void emu_buffer_read(__amdgpu_buffer_rsrc_t r, int off, int n, uint32_t* out)
{
    for (int k = 0; k < n; ++k) {
        const uint64_t o = (uint64_t)(uint32_t)off + 4ull * k;
        if (o + 4 > r.num_records) {
            out[k] = 0;
        } else {
            std::memcpy(&out[k], r.base + o, 4);  // ASan checks the allocation
        }
    }
}

typedef unsigned int emu_u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int emu_u32x4 __attribute__((ext_vector_type(4)));

// The scalar offset adds to the byte offset; the range check here takes the
// sum (stricter than a check of the vector offset alone), so an access the
// kernel relies on must be in range either way.
inline unsigned __builtin_amdgcn_raw_buffer_load_b32(__amdgpu_buffer_rsrc_t r, int off, int soff, int aux)
{
    assert(soff >= 0 && aux == 0);
    uint32_t v;
    emu_buffer_read(r, (int)((uint32_t)off + (uint32_t)soff), 1, &v);
    return v;
}

// A store outside num_records is dropped.
inline void __builtin_amdgcn_raw_buffer_store_b32(unsigned v, __amdgpu_buffer_rsrc_t r, int off, int soff, int aux)
{
    assert(soff >= 0 && aux == 0);
    const uint64_t o = (uint64_t)(uint32_t)off + (uint64_t)(uint32_t)soff;
    if (o + 4 <= r.num_records)
        std::memcpy(const_cast<char*>(r.base) + o, &v, 4);  // ASan checks the allocation
}

// Each dword of a two-dword store is range-checked on its own.
template <class V2>
inline void __builtin_amdgcn_raw_buffer_store_b64(V2 v, __amdgpu_buffer_rsrc_t r, int off, int soff, int aux)
{
    assert(soff >= 0 && aux == 0 && (off & 3) == 0);
    __builtin_amdgcn_raw_buffer_store_b32(v[0], r, off, soff, aux);
    __builtin_amdgcn_raw_buffer_store_b32(v[1], r, off + 4, soff, aux);
}

inline void __builtin_amdgcn_sched_barrier(int) {}

inline emu_u32x2 __builtin_amdgcn_raw_buffer_load_b64(__amdgpu_buffer_rsrc_t r, int off, int soff, int aux)
{
    assert(soff == 0 && aux == 0 && (off & 3) == 0);  // any dword offset, as on gfx9
    uint32_t v[2];
    emu_buffer_read(r, off, 2, v);
    return emu_u32x2{v[0], v[1]};
}

inline emu_u32x4 __builtin_amdgcn_raw_buffer_load_b128(__amdgpu_buffer_rsrc_t r, int off, int soff, int aux)
{
    assert(soff == 0 && aux == 0 && (off & 3) == 0);  // any dword offset, as on gfx9
    uint32_t v[4];
    emu_buffer_read(r, off, 4, v);
    return emu_u32x4{v[0], v[1], v[2], v[3]};
}

template <class T>
inline void emu_nontemporal_store(T v, T* p)
{
    // A gfx9-family store of several dwords needs only dword alignment: the
    // kernels store four-wide at any dword boundary of a row.
    assert(reinterpret_cast<uintptr_t>(p) % 4 == 0);
    std::memcpy(static_cast<void*>(p), &v, sizeof(T));
}
#define __builtin_nontemporal_store(v, p) emu_nontemporal_store(v, p)

// Every lane of a workgroup holds the same value wherever the kernels use it.
inline int __builtin_amdgcn_readfirstlane(int v) { return v; }
