// Host-side driver for the BVH builder tests: reads a mesh (int32 nv, nt;
// float32 pos[nv][3]; int32 idx[nt][3]) from argv[1], builds the wide BVH and
// writes int32 depth, stack, n_nodes, ok; the nodes (128 bytes each); the
// leaf order (int32 [nt]) to argv[2].
#include <cstdio>
#include <vector>

#include "../paper_1912_05494_amd/csrc/bvh_build.hpp"

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 3;
    int32_t nv = 0, nt = 0;
    if (std::fread(&nv, 4, 1, f) != 1 || std::fread(&nt, 4, 1, f) != 1) return 4;
    std::vector<float> pos(3 * (size_t)nv);
    std::vector<int32_t> idx(3 * (size_t)nt);
    if (std::fread(pos.data(), 4, pos.size(), f) != pos.size()) return 5;
    if (std::fread(idx.data(), 4, idx.size(), f) != idx.size()) return 6;
    std::fclose(f);
    const sdm::BvhResult r = sdm::build_bvh(pos.data(), nv, idx.data(), nt);
    FILE *o = std::fopen(argv[2], "wb");
    if (!o) return 7;
    const int32_t head[4] = {r.depth, r.stack, (int32_t)r.nodes.size(), r.ok ? 1 : 0};
    std::fwrite(head, 4, 4, o);
    std::fwrite(r.nodes.data(), sizeof(sdm::BvhNode), r.nodes.size(), o);
    std::fwrite(r.order.data(), 4, r.order.size(), o);
    std::fclose(o);
    return 0;
}
