// Host-only reference for the Philox4x32-10 pin: runs rocRAND's
// host-callable philox4x32_10_engine::ten_rounds (a library built from its
// published source, used as a black box) over (counter, key) records.
// Input file: n records of 6 uint32 (c0 c1 c2 c3 k0 k1); output: n x 4 uint32.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdint>
#include <vector>

// ten_rounds is a protected member; a derived class makes it callable.
struct PhiloxRounds : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *fi = std::fopen(argv[1], "rb");
    if (!fi) return 3;
    std::vector<uint32_t> in;
    uint32_t buf[6];
    while (std::fread(buf, sizeof(uint32_t), 6, fi) == 6) in.insert(in.end(), buf, buf + 6);
    std::fclose(fi);
    size_t n = in.size() / 6;
    std::vector<uint32_t> out(4 * n);
    PhiloxRounds eng;
    for (size_t i = 0; i < n; ++i) {
        uint4 c{in[6 * i], in[6 * i + 1], in[6 * i + 2], in[6 * i + 3]};
        uint2 k{in[6 * i + 4], in[6 * i + 5]};
        uint4 r = eng.ten_rounds(c, k);
        out[4 * i] = r.x; out[4 * i + 1] = r.y; out[4 * i + 2] = r.z; out[4 * i + 3] = r.w;
    }
    FILE *fo = std::fopen(argv[2], "wb");
    if (!fo) return 4;
    std::fwrite(out.data(), sizeof(uint32_t), out.size(), fo);
    std::fclose(fo);
    return 0;
}
