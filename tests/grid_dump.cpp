// Host-side driver for the sun-grid tests: reads a mesh (int32 nv, nt;
// float32 pos[nv][3]; int32 idx[nt][3]; float32 sun[3]; float64 extent) from
// argv[1], builds the grid over the triangles in input order and writes to
// argv[2]: int32 use, nx, ny; float32 e1[3], e2[3], u0, v0, idu, idv, marg;
// int32 start[nx*ny+1]; then the 48-byte candidates (all materials opaque).
#include <cstdio>
#include <vector>

#include "../paper_1912_05494_amd/csrc/sun_grid.hpp"

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 3;
    int32_t nv = 0, nt = 0;
    if (std::fread(&nv, 4, 1, f) != 1 || std::fread(&nt, 4, 1, f) != 1) return 4;
    std::vector<float> pos(3 * (size_t)nv);
    std::vector<int32_t> idx(3 * (size_t)nt);
    float sun[3];
    double extent = 0.0;
    if (std::fread(pos.data(), 4, pos.size(), f) != pos.size()) return 5;
    if (std::fread(idx.data(), 4, idx.size(), f) != idx.size()) return 6;
    if (std::fread(sun, 4, 3, f) != 3 || std::fread(&extent, 8, 1, f) != 1) return 7;
    std::fclose(f);
    std::vector<sdm::TriDev> tris(nt);
    for (int32_t t = 0; t < nt; ++t) {
        const float *p[3];
        for (int c = 0; c < 3; ++c) p[c] = pos.data() + 3 * (size_t)idx[3 * (size_t)t + c];
        tris[t].a = make_float4(p[0][0], p[0][1], p[0][2], 0.0f);
        tris[t].b = make_float4(p[1][0], p[1][1], p[1][2], 0.0f);
        tris[t].c = make_float4(p[2][0], p[2][1], p[2][2], 0.0f);
    }
    const int32_t mat_type[1] = {0};
    const sdm::SunGrid g = sdm::build_sun_grid(tris.data(), nt, mat_type, sun, extent);
    FILE *o = std::fopen(argv[2], "wb");
    if (!o) return 8;
    const int32_t head[3] = {g.use ? 1 : 0, g.nx, g.ny};
    std::fwrite(head, 4, 3, o);
    const float par[11] = {g.e1[0], g.e1[1], g.e1[2], g.e2[0], g.e2[1], g.e2[2], g.u0, g.v0, g.idu, g.idv, g.marg};
    std::fwrite(par, 4, 11, o);
    std::fwrite(g.start.data(), 4, g.start.size(), o);
    std::fwrite(g.cand.data(), sizeof(sdm::GridCand), g.cand.size(), o);
    std::fclose(o);
    return 0;
}
