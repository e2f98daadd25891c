// Host check of the population layouts (kbc::Geom, pop_index): for the
// x-blocked layout and for planes with and without a gap, every (slot, x, y,
// z) maps to a distinct element inside the extent the buffer is allocated
// with; the blocked layout fills its extent exactly and keeps the 27 slots of
// a chunk of B nodes adjacent in x contiguous; a slot's span is what the
// step kernels address with 32-bit offsets.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "kbc_internal.h"

using namespace kbc;

static long check(Geom g, bool blocked, uint64_t pad)
{
    long bad = 0;
    if (blocked) geom_blocked(g);
    else geom_planes(g, pad);
    const uint64_t ext = geom_extent(g);
    std::vector<uint8_t> seen(ext, 0);
    uint64_t slot0_max = 0;
    for (int s = 0; s < 27; ++s)
        for (uint32_t z = 0; z < g.nz; ++z)
            for (uint32_t y = 0; y < g.ny; ++y)
                for (uint32_t x = 0; x < g.nx; ++x) {
                    const uint64_t i = pop_index(g, s, x, y, z);
                    if (i >= ext) {
                        ++bad;
                        continue;
                    }
                    if (seen[i]++) ++bad;
                    if (s == 0 && i + 1 > slot0_max) slot0_max = i + 1;
                }
    uint64_t used = 0;
    for (uint8_t v : seen) used += v;
    if (used != 27ull * g.nnodes) ++bad;
    if (blocked && used != ext) ++bad;               // no holes
    if (!blocked && ext != 26 * g.plane + g.nnodes) ++bad;
    if (geom_slot_span_bytes(g, 4) != slot0_max * 4) ++bad;
    if (geom_is_planes(g) == blocked) ++bad;
    if (blocked) {
        // the 27 slots of a chunk of B nodes along x are one contiguous run
        const uint32_t B = (uint32_t)g.plane;
        if (g.nx % B) ++bad;
        for (uint32_t z = 0; z < g.nz; ++z)
            for (uint32_t y = 0; y < g.ny; ++y)
                for (uint32_t x0 = 0; x0 < g.nx; x0 += B) {
                    const uint64_t base = pop_index(g, 0, x0, y, z);
                    for (int s = 0; s < 27; ++s)
                        for (uint32_t k = 0; k < B; ++k)
                            if (pop_index(g, s, x0 + k, y, z) != base + (uint64_t)s * B + k) ++bad;
                }
    }
    return bad;
}

int main()
{
    const uint32_t nxs[] = {1, 2, 13, 24, 32, 33, 64, 96, 100, 128, 192, 256};
    const uint32_t yzs[][2] = {{1, 1}, {3, 2}, {5, 4}};
    long bad = 0;
    int cases = 0;
    for (uint32_t nx : nxs)
        for (auto& yz : yzs) {
            Geom g{};
            g.nx = nx;
            g.ny = yz[0];
            g.nz = yz[1];
            g.nnodes = nx * yz[0] * yz[1];
            bad += check(g, true, 0);
            bad += check(g, false, 0);
            bad += check(g, false, 7);
            cases += 3;
        }
    // chunk sizes the blocked layout picks
    Geom g{};
    g.nx = 192; g.ny = 1; g.nz = 1; g.nnodes = 192;
    geom_blocked(g);
    if (g.plane != 64 || g.xshift != 6) ++bad;
    g.nx = 96; g.nnodes = 96;
    geom_blocked(g);
    if (g.plane != 32 || g.xshift != 5) ++bad;
    g.nx = 100; g.nnodes = 100;
    geom_blocked(g);
    if (g.plane != 100 || g.xshift != 31) ++bad;
    std::printf("%d layouts checked, %ld mismatches\n", cases, bad);
    return bad == 0 ? 0 : 1;
}
