// Runs the multi-filter persistent kernel (CONV_BATCH=2) on the CPU (see
// hip_emu.h) over images of several filter sizes, with the descriptor, owner
// and counter tables laid out as the host library lays them out: problems in
// group order, each group's tiles contiguous. Runs the launch twice (outputs
// reset in between) and checks that the tile counters are back at 0 after each.
// Usage: emu_multi GRID DIR N H0 W0 G0 H1 W1 G1 ...   (G = group index; DIR
// holds in<k>.f32, f<k>.f32; writes out<k>.f32)
#include "hip_emu.h"

#include <algorithm>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

thread_local emu_dim3 threadIdx;
thread_local emu_dim3 blockIdx;
emu_dim3 blockDim;
emu_dim3 gridDim;
std::barrier<>* emu_block_barrier;

#include "../../paper_2407_11488_amd/csrc/conv2d_direct.hip"

struct GroupShape {
    int fh, fw, bx, by, tx, ty;
};
#define G(k, fh, fw, bx, by, tx, ty, lds, unr) GroupShape{fh, fw, bx, by, tx, ty},
static const GroupShape kGroups[] = {CONV_GROUPS};
#undef G

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
    std::vector<int> H(n), W(n), grp(n);
    for (int k = 0; k < n; ++k) {
        H[k] = std::atoi(argv[4 + 3 * k]);
        W[k] = std::atoi(argv[5 + 3 * k]);
        grp[k] = std::atoi(argv[6 + 3 * k]);
    }
    // Descriptor order: by group, then by problem number.
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return grp[a] < grp[b]; });
    std::vector<ConvDesc> descs(n);
    std::vector<unsigned short> owner;
    std::vector<float*> outs(n);
    int total = 0;
    for (int slot = 0; slot < n; ++slot) {
        const int k = order[slot];
        const GroupShape& g = kGroups[grp[k]];
        const size_t n_in = (size_t)(H[k] + g.fh - 1) * (W[k] + g.fw - 1);
        ConvDesc& d = descs[slot];
        d.in = read_exact(dir + "/in" + std::to_string(k) + ".f32", n_in);
        d.filt = read_exact(dir + "/f" + std::to_string(k) + ".f32", (size_t)g.fh * g.fw);
        outs[k] = static_cast<float*>(std::aligned_alloc(16, (((size_t)H[k] * W[k] * 4 + 15) / 16) * 16));
        d.out = outs[k];
        d.H = H[k];
        d.W = W[k];
        const int tw = g.bx * g.tx, th = g.by * g.ty;
        d.tiles_x = (W[k] + tw - 1) / tw;
        d.n_tiles = d.tiles_x * ((H[k] + th - 1) / th);
        d.tile_begin = total;
        d.in_bytes = (unsigned)(n_in * 4);
        d.group = grp[k];
        total += d.n_tiles;
        owner.insert(owner.end(), (size_t)d.n_tiles, (unsigned short)slot);
    }
    if (grid > total) { std::fprintf(stderr, "grid above the tile count\n"); return 2; }
    int counters[2] = {0, 0};
    blockDim = {CONV_NT, 1, 1};
    gridDim = {(unsigned)grid, 1, 1};
    for (int launch = 0; launch < 2; ++launch) {
        for (int k = 0; k < n; ++k)
            for (size_t e = 0; e < (size_t)H[k] * W[k]; ++e) outs[k][e] = std::nanf("");
        for (int b = 0; b < grid; ++b) {
            std::barrier<> bar(CONV_NT);
            emu_block_barrier = &bar;
            std::vector<std::thread> th_;
            for (int t = 0; t < CONV_NT; ++t)
                th_.emplace_back([&, t, b] {
                    threadIdx = {(unsigned)t, 0, 0};
                    blockIdx = {(unsigned)b, 0, 0};
                    CONV_NAME(descs.data(), owner.data(), total, counters);
                });
            for (auto& x : th_) x.join();
        }
        if (counters[0] != 0 || counters[1] != 0) {
            std::fprintf(stderr, "tile counters not reset after launch %d: %d %d\n", launch, counters[0], counters[1]);
            return 3;
        }
    }
    for (int k = 0; k < n; ++k) {
        FILE* o = std::fopen((dir + "/out" + std::to_string(k) + ".f32").c_str(), "wb");
        std::fwrite(outs[k], 4, (size_t)H[k] * W[k], o);
        std::fclose(o);
        std::free(outs[k]);
    }
    for (auto& d : descs) {
        std::free((void*)d.in);
        std::free((void*)d.filt);
    }
    return 0;
}
