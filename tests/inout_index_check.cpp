// Host check of the in/out index (paper_2106_12863_amd/csrc/inout_index.h):
// the index built from a union's boundaries U answers membership = parity of
// the number of boundaries <= a (the union starts outside at address 0), for
// random unions that put many boundaries into few /16 blocks (slot overflow
// lists), crowd the start of blocks, or spread over the whole space, plus
// boundaries at a block's first address and at the top of the space.
// Addresses: uniform, and each boundary +-2.  Exit status 0 when every
// lookup agrees.
#include "inout_index.h"
#include <cstdio>
#include <random>
#include <algorithm>
using namespace sinet;
int main() {
    std::mt19937_64 rng(5);
    long bad = 0, checked = 0;
    for (int trial = 0; trial < 60; ++trial) {
        std::vector<uint32_t> U;
        int nb = (trial % 6 == 0) ? 5000 : 200 + (int)(rng() % 3000);
        for (int i = 0; i < nb; ++i) {
            uint32_t v;
            if (trial % 3 == 0) v = (uint32_t)(rng() % 65536) << 16 | (uint32_t)(rng() % 4096);  // dense in few blocks
            else if (trial % 3 == 1) v = (uint32_t)((rng() % 40) << 16) | (uint32_t)(rng() & 0xFFFF); // many per block
            else v = (uint32_t)rng();
            if (v == 0) continue;
            U.push_back(v);
        }
        if (trial == 7) { U.push_back(0xFFFFFFFFu); U.push_back(0x00010000u); U.push_back(0xFFFF0000u); }
        std::sort(U.begin(), U.end());
        U.erase(std::unique(U.begin(), U.end()), U.end());
        std::vector<uint32_t> io; IoLayout lay{};
        if (!build_inout_index(U, io, lay)) { printf("build failed\n"); return 1; }
        io.resize(io.size() + 4, 0);
        auto truth = [&](uint32_t a) { return (uint32_t)((std::upper_bound(U.begin(), U.end(), a) - U.begin()) & 1); };
        for (int k = 0; k < 200000; ++k) {
            uint32_t a[8], in[8];
            for (int q = 0; q < 8; ++q) {
                uint64_t r = rng();
                if (r % 3 == 0 && !U.empty()) { uint32_t b = U[rng() % U.size()]; a[q] = b + (uint32_t)(int)(rng() % 5) - 2; }
                else a[q] = (uint32_t)r;
            }
            inout_lookup<8>(io.data(), lay.slot, lay.list, a, in);
            for (int q = 0; q < 8; ++q) { ++checked; if (in[q] != truth(a[q])) { if (bad < 5) printf("bad trial %d a=%08x got %u want %u\n", trial, a[q], in[q], truth(a[q])); ++bad; } }
        }
    }
    printf("checked %ld bad %ld\n", checked, bad);
    return bad != 0;
}
