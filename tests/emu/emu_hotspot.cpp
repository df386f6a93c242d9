// Runs the hotspot kernel (hotspot.hip) on the CPU (see hip_emu.h): the
// launches of one run of `steps` steps, alternating between two buffers as
// the host library does, every workgroup's threads as host threads.
// Usage: emu_hotspot ROWS COLS STEPS CC GX GY GZ TAMB DIR  (DIR holds temp.f32
// and power.f32; writes out.f32)
#include "hip_emu.h"

#include <memory>
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

#include "../../paper_2407_11488_amd/csrc/hotspot.hip"

static std::vector<float> read_all(const std::string& path, size_t n)
{
    std::vector<float> v(n);
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f || std::fread(v.data(), 4, n, f) != n) { std::fprintf(stderr, "read %s failed\n", path.c_str()); std::exit(2); }
    std::fclose(f);
    return v;
}

int main(int argc, char** argv)
{
    if (argc != 10) return 2;
    const int rows = std::atoi(argv[1]), cols = std::atoi(argv[2]), steps = std::atoi(argv[3]);
    const float cc = std::strtof(argv[4], nullptr), gx = std::strtof(argv[5], nullptr);
    const float gy = std::strtof(argv[6], nullptr), gz = std::strtof(argv[7], nullptr);
    const float ta = std::strtof(argv[8], nullptr);
    // The step's coefficients grouped by term, as the library's host code
    // passes them: computed in double, rounded once.
    const float ka = (float)(1.0 - (double)cc * (2.0 * gx + 2.0 * gy + gz));
    const float ky = (float)((double)cc * gy), kx = (float)((double)cc * gx);
    const float q = (float)((double)cc * gz * ta);
    const std::string dir = argv[9];
    const size_t n = (size_t)rows * cols;
    std::vector<float> temp = read_all(dir + "/temp.f32", n), power = read_all(dir + "/power.f32", n);
    std::vector<float> a(n, std::nanf("")), b(n, std::nanf(""));
    const int tiles_x = (cols + OW - 1) / OW, tiles_y = (rows + OH - 1) / OH, n_tiles = tiles_x * tiles_y;
    const int launches = (steps + HS_TT - 1) / HS_TT;
    const float* src = temp.data();
    blockDim = {HS_NT, 1, 1};
    gridDim = {(unsigned)n_tiles, 1, 1};
    for (int i = 0; i < launches; ++i) {
        float* dst = ((launches - 1 - i) % 2 == 0) ? a.data() : b.data();
        const int this_steps = std::min(HS_TT, steps - i * HS_TT);
        for (int g = 0; g < n_tiles; ++g) {
            std::barrier<> bar(HS_NT);
            emu_block_barrier = &bar;
            std::vector<int> dpp(HS_NT);
            emu_dpp_slots = dpp.data();
            std::vector<std::unique_ptr<std::barrier<>>> waves;
            std::vector<std::barrier<>*> wave_ptrs;
            for (int w0 = 0; w0 < HS_NT; w0 += 64) {
                waves.emplace_back(new std::barrier<>(std::min(64, HS_NT - w0)));
                wave_ptrs.push_back(waves.back().get());
            }
            emu_wave_barriers = wave_ptrs.data();
            std::vector<std::thread> th;
            for (int t = 0; t < HS_NT; ++t)
                th.emplace_back([&, t, g] {
                    threadIdx = {(unsigned)t, 0, 0};
                    blockIdx = {(unsigned)g, 0, 0};
                    HS_NAME(src, power.data(), dst, rows, cols, this_steps, tiles_x, n_tiles, ka, ky, kx, cc, q);
                });
            for (auto& x : th) x.join();
        }
        src = dst;
    }
    FILE* o = std::fopen((dir + "/out.f32").c_str(), "wb");
    std::fwrite(launches ? a.data() : temp.data(), 4, n, o);
    std::fclose(o);
    return 0;
}
