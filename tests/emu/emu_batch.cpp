// Runs the persistent batched kernel (CONV_BATCH=1) on the CPU (see
// hip_emu.h) over several images of one filter size, with the descriptor and
// tile-owner tables laid out as the host library lays them out.
// Usage: emu_batch GRID DIR N H0 W0 H1 W1 ...   (DIR holds in<k>.f32, f<k>.f32;
// writes out<k>.f32)
#include "hip_emu.h"

#include <string>
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

static float* read_exact(const std::string& path, size_t n)
{
    float* p = static_cast<float*>(std::aligned_alloc(16, ((n * 4 + 15) / 16) * 16));
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f || std::fread(p, 4, n, f) != n) { std::fprintf(stderr, "read %s failed\n", path.c_str()); std::exit(2); }
    std::fclose(f);
    return p;
}

int main(int argc, char** argv)
{
    const int grid = std::atoi(argv[1]);
    const std::string dir = argv[2];
    const int n = std::atoi(argv[3]);
    std::vector<ConvDesc> descs(n);
    std::vector<unsigned short> owner;
    std::vector<float*> outs(n);
    std::vector<size_t> out_n(n);
    int total = 0;
    for (int k = 0; k < n; ++k) {
        const int H = std::atoi(argv[4 + 2 * k]), W = std::atoi(argv[5 + 2 * k]);
        const size_t n_in = (size_t)(H + CONV_FH - 1) * (W + CONV_FW - 1);
        ConvDesc& d = descs[k];
        d.in = read_exact(dir + "/in" + std::to_string(k) + ".f32", n_in);
        d.filt = read_exact(dir + "/f" + std::to_string(k) + ".f32", (size_t)CONV_FH * CONV_FW);
        out_n[k] = (size_t)H * W;
        outs[k] = static_cast<float*>(std::aligned_alloc(16, ((out_n[k] * 4 + 15) / 16) * 16));
        for (size_t e = 0; e < out_n[k]; ++e) outs[k][e] = std::nanf("");
        d.out = outs[k];
        d.H = H;
        d.W = W;
        const int tw = CONV_BX * CONV_TX, th = CONV_BY * CONV_TY;
        d.tiles_x = (W + tw - 1) / tw;
        const int tiles = d.tiles_x * ((H + th - 1) / th);
        d.tile_begin = total;
        d.in_bytes = (unsigned)(n_in * 4);
        d.n_tiles = tiles;
        total += tiles;
        owner.insert(owner.end(), (size_t)tiles, (unsigned short)k);
    }
    blockDim = {CONV_BX * CONV_BY, 1, 1};
    gridDim = {(unsigned)grid, 1, 1};
    for (int b = 0; b < grid; ++b) {
        std::barrier<> bar(CONV_BX * CONV_BY);
        emu_block_barrier = &bar;
        std::vector<std::thread> th_;
        for (int t = 0; t < CONV_BX * CONV_BY; ++t)
            th_.emplace_back([&, t, b] {
                threadIdx = {(unsigned)t, 0, 0};
                blockIdx = {(unsigned)b, 0, 0};
                CONV_NAME(descs.data(), owner.data(), total);
            });
        for (auto& x : th_) x.join();
    }
    for (int k = 0; k < n; ++k) {
        FILE* o = std::fopen((dir + "/out" + std::to_string(k) + ".f32").c_str(), "wb");
        std::fwrite(outs[k], 4, out_n[k], o);
        std::fclose(o);
        std::free(outs[k]);
        std::free((void*)descs[k].in);
        std::free((void*)descs[k].filt);
    }
    return 0;
}
