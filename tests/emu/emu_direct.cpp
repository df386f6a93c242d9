// Runs the tunable direct-convolution kernel source on the CPU (see
// hip_emu.h): every workgroup of the launch the library would make, one host
// thread per GPU thread. Usage: emu_direct in.f32 filt.f32 out.f32 H W
// Input/filter/output are raw little-endian FP32 files of the exact sizes.
#include "hip_emu.h"

#include <thread>
#include <vector>

thread_local emu_dim3 threadIdx;
thread_local emu_dim3 blockIdx;
emu_dim3 blockDim;
emu_dim3 gridDim;
std::barrier<>* emu_block_barrier;
int* emu_dpp_slots;
std::barrier<>** emu_wave_barriers;

#include "../../paper_2407_11488_amd/csrc/conv2d_direct.hip"

static std::vector<float> read_f32(const char* path, size_t n)
{
    std::vector<float> v(n);
    FILE* f = std::fopen(path, "rb");
    if (!f || std::fread(v.data(), 4, n, f) != n) { std::fprintf(stderr, "read %s failed\n", path); std::exit(2); }
    std::fclose(f);
    return v;
}

int main(int argc, char** argv)
{
    if (argc != 6) { std::fprintf(stderr, "usage\n"); return 2; }
    const int H = std::atoi(argv[4]), W = std::atoi(argv[5]);
    const long long P = (long long)W + CONV_FW - 1;
    const size_t n_in = (size_t)(H + CONV_FH - 1) * P;
    std::vector<float> in = read_f32(argv[1], n_in);
    std::vector<float> f = read_f32(argv[2], (size_t)CONV_FH * CONV_FW);
    // Exact-size heap copies so that AddressSanitizer sees every overrun.
    float* d_in = static_cast<float*>(std::aligned_alloc(16, ((n_in * 4 + 15) / 16) * 16));
    std::memcpy(d_in, in.data(), n_in * 4);
    float* d_f = new float[(size_t)CONV_FH * CONV_FW];
    std::memcpy(d_f, f.data(), f.size() * 4);
    float* d_out = static_cast<float*>(std::aligned_alloc(16, (((size_t)H * W * 4 + 15) / 16) * 16));
    for (size_t k = 0; k < (size_t)H * W; ++k) d_out[k] = std::nanf("");
#if CONV_FCONST
    std::memcpy(conv_filter, d_f, sizeof conv_filter);
#endif
    // One band (the tests use small images); same arguments as the library.
    const int tw = CONV_BX * CONV_TX, th = CONV_BY * CONV_TY;
    const int tiles_x = (W + tw - 1) / tw, tiles_y = (H + th - 1) / th, n_tiles = tiles_x * tiles_y;
    const unsigned in_bytes = (unsigned)(n_in * 4);
    blockDim = {CONV_BX * CONV_BY, 1, 1};
    gridDim = {(unsigned)n_tiles, 1, 1};
    for (int b = 0; b < n_tiles; ++b) {
        std::barrier<> bar(CONV_BX * CONV_BY);
        emu_block_barrier = &bar;
        std::vector<std::thread> th_;
        for (int t = 0; t < CONV_BX * CONV_BY; ++t)
            th_.emplace_back([=] {
                threadIdx = {(unsigned)t, 0, 0};
                blockIdx = {(unsigned)b, 0, 0};
                CONV_NAME(d_in, d_f, d_out, H, W, tiles_x, n_tiles, in_bytes);
            });
        for (auto& x : th_) x.join();
    }
    FILE* o = std::fopen(argv[3], "wb");
    std::fwrite(d_out, 4, (size_t)H * W, o);
    std::fclose(o);
    std::free(d_in);
    std::free(d_out);
    delete[] d_f;
    return 0;
}
