// Host-side check of the shared-node enumeration and partial-slot arithmetic
// used by the assembly kernels (compiled with hipcc, runs on the CPU only).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <tuple>
#include <vector>

#include "../../paper_2401_07805_amd/csrc/shared_nodes.h"

using namespace vpp;

static int fails = 0;
#define CHECK(c, ...)                                   \
    do {                                                \
        if (!(c)) {                                     \
            if (fails < 20) std::printf(__VA_ARGS__);   \
            ++fails;                                    \
        }                                               \
    } while (0)

static void check(int k, const int (&nc)[3], const int (&tile)[3], int bcmask)
{
    MeshArgs m{};
    for (int d = 0; d < 3; ++d) {
        m.nc[d] = nc[d];
        m.nn[d] = k * nc[d] + 1;
        m.ntile[d] = (nc[d] + tile[d] - 1) / tile[d];
    }
    m.bcmask = bcmask;
    // brute force: node shared iff it lies in two tiles along some direction
    std::set<std::tuple<int, int, int>> ref;
    for (int l = 0; l < m.nn[2]; ++l)
        for (int j = 0; j < m.nn[1]; ++j)
            for (int i = 0; i < m.nn[0]; ++i) {
                const int idx[3] = {i, j, l};
                bool sh = false;
                for (int d = 0; d < 3; ++d) {
                    const int s = k * tile[d];
                    if (idx[d] % s == 0 && idx[d] / s > 0 && idx[d] / s < m.ntile[d]) sh = true;
                }
                if (sh) ref.insert({i, j, l});
            }
    const SharedEnum e = shared_enum(m, k, tile);
    const int64_t total = e.cz + e.cy + e.cx;
    CHECK(total == (int64_t)ref.size(), "count k=%d nc=%d,%d,%d tile=%d,%d,%d: %lld vs %zu\n", k, nc[0], nc[1],
          nc[2], tile[0], tile[1], tile[2], (long long)total, ref.size());
    std::set<std::tuple<int, int, int>> got;
    const int64_t bs = (int64_t)(k * tile[0] + 1) * (k * tile[1] + 1) * (k * tile[2] + 1);
    const int64_t ntiles = (int64_t)m.ntile[0] * m.ntile[1] * m.ntile[2];
    for (int64_t f = 0; f < total; ++f) {
        int i, j, l;
        shared_node(e, f, i, j, l);
        CHECK(i >= 0 && i < m.nn[0] && j >= 0 && j < m.nn[1] && l >= 0 && l < m.nn[2],
              "out of range f=%lld -> %d %d %d\n", (long long)f, i, j, l);
        CHECK(got.insert({i, j, l}).second, "duplicate %d %d %d\n", i, j, l);
        CHECK(shared_index(e, i, j, l) == f, "shared_index(%d,%d,%d) = %lld, expected %lld\n", i, j, l,
              (long long)shared_index(e, i, j, l), (long long)f);
        int64_t slot[8];
        const int n = shared_slots(m, k, tile, i, j, l, slot);
        // every sharer tile has a distinct rank in [0, n) matching the slot order
        for (int c = 0; c < n; ++c) {
            const int64_t tt = slot[c] / bs;
            const int tv[3] = {(int)(tt % m.ntile[0]), (int)((tt / m.ntile[0]) % m.ntile[1]),
                               (int)(tt / ((int64_t)m.ntile[0] * m.ntile[1]))};
            int cnt, rank;
            sharer_rank(m, k, tile, i, j, l, tv, cnt, rank);
            CHECK(cnt == n && rank == c, "rank %d/%d vs slot %d/%d\n", rank, cnt, c, n);
        }
        CHECK(n >= 2 && n <= 8, "slot count %d\n", n);
        CHECK(sharer_count(e, i, j, l) == n, "sharer_count %d vs %d\n", sharer_count(e, i, j, l), n);
        for (int c = 0; c < n; ++c) {
            CHECK(slot[c] >= 0 && slot[c] < ntiles * bs, "slot out of range\n");
            // the slot's tile block contains the node at that local position
            const int64_t t = slot[c] / bs, loc = slot[c] % bs;
            const int tx = (int)(t % m.ntile[0]), ty = (int)((t / m.ntile[0]) % m.ntile[1]),
                      tz = (int)(t / ((int64_t)m.ntile[0] * m.ntile[1]));
            const int bx = k * tile[0] + 1, by = k * tile[1] + 1;
            const int lx = (int)(loc % bx), ly = (int)((loc / bx) % by), lz = (int)(loc / ((int64_t)bx * by));
            CHECK(tx * k * tile[0] + lx == i && ty * k * tile[1] + ly == j && tz * k * tile[2] + lz == l,
                  "slot decodes to another node\n");
            CHECK(lx <= k * (nc[0] - tile[0] * tx < tile[0] ? nc[0] - tile[0] * tx : tile[0]), "slot past block\n");
        }
    }
    CHECK(got == ref, "set mismatch\n");
    // node-space lookup: every node, shared or not, Dirichlet or not
    for (int l = 0; l < m.nn[2]; ++l)
        for (int j = 0; j < m.nn[1]; ++j)
            for (int i = 0; i < m.nn[0]; ++i) {
                const int g = i + m.nn[0] * (j + m.nn[1] * l);
                const bool sh = ref.count({i, j, l}) > 0 && !is_dirichlet(m, i, j, l);
                int f = -1, cnt = 0;
                const bool got_sh = shared_lookup(e, m.bcmask, g, f, cnt);
                CHECK(got_sh == sh, "shared_lookup(%d,%d,%d) = %d, expected %d\n", i, j, l, (int)got_sh, (int)sh);
                if (sh && got_sh) {
                    CHECK(f == shared_index(e, i, j, l), "shared_lookup f %d vs %lld\n", f,
                          (long long)shared_index(e, i, j, l));
                    CHECK(cnt == sharer_count(e, i, j, l), "shared_lookup count %d vs %d\n", cnt,
                          sharer_count(e, i, j, l));
                }
            }
    // the tile-side formula used by the apply kernels' write-out: every node on a
    // shared face of every tile block maps to its enumeration index and rank
    for (int tz = 0; tz < m.ntile[2]; ++tz)
        for (int ty = 0; ty < m.ntile[1]; ++ty)
            for (int tx = 0; tx < m.ntile[0]; ++tx) {
                const int tt[3] = {tx, ty, tz};
                int ext[3];
                for (int d = 0; d < 3; ++d) {
                    const int cells = nc[d] - tile[d] * tt[d] < tile[d] ? nc[d] - tile[d] * tt[d] : tile[d];
                    ext[d] = k * cells + 1;
                }
                for (int ll = 0; ll < ext[2]; ++ll)
                    for (int lj = 0; lj < ext[1]; ++lj)
                        for (int li = 0; li < ext[0]; ++li) {
                            const bool lo0 = li == 0 && tx > 0, lo1 = lj == 0 && ty > 0, lo2 = ll == 0 && tz > 0;
                            const bool hi0 = li == ext[0] - 1 && tx < m.ntile[0] - 1;
                            const bool hi1 = lj == ext[1] - 1 && ty < m.ntile[1] - 1;
                            const bool hi2 = ll == ext[2] - 1 && tz < m.ntile[2] - 1;
                            if (!(lo0 || lo1 || lo2 || hi0 || hi1 || hi2)) continue;
                            const int gi = tx * k * tile[0] + li, gj = ty * k * tile[1] + lj, gl = tz * k * tile[2] + ll;
                            int64_t ff;
                            int rank;
                            shared_from_tile(m, tt, lo0, lo1, lo2, hi0, hi1, hi2, gi, gj, gl, ff, rank);
                            CHECK(ff >= 0 && ff < total && ff == shared_index(e, gi, gj, gl),
                                  "tile-side index %lld vs %lld\n", (long long)ff, (long long)shared_index(e, gi, gj, gl));
                            int cnt, rk;
                            sharer_rank(m, k, tile, gi, gj, gl, tt, cnt, rk);
                            CHECK(rank == rk && rank >= 0 && rank < cnt, "tile-side rank %d vs %d\n", rank, rk);
                        }
            }
}

// The parity colouring of the cells (cell_color / color_cell): every cell in
// exactly one colour, and no node shared by two cells of one colour.
static void check_colors(int k, const int (&nc)[3])
{
    MeshArgs m{};
    for (int d = 0; d < 3; ++d) {
        m.nc[d] = nc[d];
        m.nn[d] = k * nc[d] + 1;
    }
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    std::vector<int> seen(ncell, 0);
    std::vector<int> owner((size_t)m.nn[0] * m.nn[1] * m.nn[2]);
    for (int c = 0; c < 8; ++c) {
        const CellColor cc = cell_color(m, c);
        std::fill(owner.begin(), owner.end(), -1);
        int cx, cy, cz;
        CHECK(!color_cell(cc, color_count(cc), cx, cy, cz), "colour %d: position past the end accepted\n", c);
        for (int64_t i = 0; i < color_count(cc); ++i) {
            if (!color_cell(cc, i, cx, cy, cz)) {
                CHECK(false, "colour %d: position %lld rejected\n", c, (long long)i);
                continue;
            }
            const bool in = cx >= 0 && cx < nc[0] && cy >= 0 && cy < nc[1] && cz >= 0 && cz < nc[2];
            CHECK(in, "colour %d: cell (%d %d %d) outside the mesh\n", c, cx, cy, cz);
            if (!in) continue;
            CHECK(((cx & 1) | ((cy & 1) << 1) | ((cz & 1) << 2)) == c, "cell (%d %d %d) in colour %d\n", cx, cy, cz, c);
            ++seen[cx + (int64_t)nc[0] * (cy + (int64_t)nc[1] * cz)];
            const int id = (int)(cx + nc[0] * (cy + nc[1] * cz));
            for (int a2 = 0; a2 <= k; ++a2)
                for (int a1 = 0; a1 <= k; ++a1)
                    for (int a0 = 0; a0 <= k; ++a0) {
                        const int64_t g = node_index(m, k * cx + a0, k * cy + a1, k * cz + a2);
                        CHECK(owner[g] < 0, "colour %d: node %lld in cells %d and %d\n", c, (long long)g, owner[g], id);
                        owner[g] = id;
                    }
        }
    }
    for (int64_t i = 0; i < ncell; ++i) CHECK(seen[i] == 1, "cell %lld in %d colours\n", (long long)i, seen[i]);
}

int main()
{
    const int tiles[][3] = {{8, 8, 4}, {16, 4, 4}, {8, 4, 4}, {32, 2, 2}, {4, 4, 2}, {4, 2, 2}, {8, 2, 2},
                            {2, 2, 2}, {4, 4, 1}, {1, 1, 1}, {3, 5, 2}};
    const int sizes[][3] = {{1, 1, 1}, {2, 3, 1}, {5, 4, 3}, {8, 8, 8}, {9, 5, 7}, {16, 16, 16}, {13, 7, 11},
                            {33, 4, 5}, {17, 17, 2}, {6, 40, 3}};
    int ncase = 0;
    for (int k = 2; k <= 4; ++k)
        for (const auto& t : tiles)
            for (const auto& s : sizes) {
                check(k, s, t, (ncase % 3 == 0) ? 63 : (ncase % 3 == 1 ? 0 : 21));
                ++ncase;
            }
    for (int k = 1; k <= 4; ++k)
        for (const auto& sz : sizes) {
            check_colors(k, sz);
            ++ncase;
        }
    std::printf("%d cases, %d failures\n", ncase, fails);
    return fails ? 1 : 0;
}
