// Host program used only by the tests: evaluates Philox4x32-10 with the
// engine of the rocRAND source header shipped with ROCm, an implementation
// written independently of both this repository's oracle and its kernels.
// Reads records of six uint32 (counter words 0..3, key words 0..1) from the
// file named by argv[1] and writes four uint32 per record (the ten-round
// output) to the file named by argv[2].
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdint>
#include <cstdio>
#include <vector>

// ten_rounds() is a protected member of the engine; a derived class exposes it.
struct Philox : rocrand_device::philox4x32_10_engine {
    uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main(int argc, char** argv)
{
    if (argc != 3) {
        std::fprintf(stderr, "usage: %s in.bin out.bin\n", argv[0]);
        return 2;
    }
    std::FILE* fi = std::fopen(argv[1], "rb");
    if (!fi) return 3;
    std::vector<uint32_t> in;
    uint32_t rec[6];
    while (std::fread(rec, sizeof rec, 1, fi) == 1) in.insert(in.end(), rec, rec + 6);
    std::fclose(fi);
    const size_t n = in.size() / 6;
    std::vector<uint32_t> out(4 * n);
    Philox eng;
    for (size_t i = 0; i < n; ++i) {
        const uint32_t* r = &in[6 * i];
        uint4 c;
        c.x = r[0];
        c.y = r[1];
        c.z = r[2];
        c.w = r[3];
        uint2 k;
        k.x = r[4];
        k.y = r[5];
        const uint4 o = eng.rounds(c, k);
        out[4 * i + 0] = o.x;
        out[4 * i + 1] = o.y;
        out[4 * i + 2] = o.z;
        out[4 * i + 3] = o.w;
    }
    std::FILE* fo = std::fopen(argv[2], "wb");
    if (!fo) return 4;
    const size_t wrote = std::fwrite(out.data(), sizeof(uint32_t), out.size(), fo);
    std::fclose(fo);
    return wrote == out.size() ? 0 : 5;
}
