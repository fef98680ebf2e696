// Host-side bounds check of the fused stage kernel's index scheme (no GPU use).
//
// For every tile shape the kernels are instantiated with, and a set of grid
// sizes and boundary kinds, enumerate exactly the indices k_stage computes:
// the staging plan (cross region -> per-direction line arrays in LDS), the
// 6-cell stencils of every face, the face slots of every owned cell, and the
// ghost-cell map of every global load.  Exit status 0 only if every index is
// in bounds and points at the intended cell.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <tuple>

#include "stage_kernel.hpp"

using namespace bub;

static int failures = 0;
#define CHECK(cond, ...)                                 \
    do {                                                 \
        if (!(cond)) {                                   \
            if (failures < 20) std::printf(__VA_ARGS__); \
            ++failures;                                  \
        }                                                \
    } while (0)

template <int D, int TX, int TY, int TZ>
void check_tile()
{
    using G = Geo<D, TX, TY, TZ>;
    // 1) staging plan: slot -> cell; every slot in range and written once
    std::map<int, std::tuple<int, int, int>> slot_cell;
    for (int ci = 0; ci < G::C; ++ci) {
        int i, j, k;
        int h = G::cdecode(ci, i, j, k);
        int out = (i < 0 || i >= G::TX) + (j < 0 || j >= G::TY) + (k < 0 || k >= G::TZ);
        CHECK(out == (h >= 0 ? 1 : 0), "D%d ci %d halo kind\n", D, ci);
        CHECK(i >= -3 && i < G::TX + 3 && j >= -3 && j < G::TY + 3 && k >= -3 && k < G::TZ + 3, "range\n");
        int slots[3] = {-1, -1, -1};
        if (h == 0 || h < 0) slots[0] = G::template lidx<0>(i, j, k);
        if (D > 1 && (h == 1 || h < 0)) slots[1] = G::template lidx<(D > 1 ? 1 : 0)>(i, j, k);
        if (D > 2 && (h == 2 || h < 0)) slots[2] = G::template lidx<(D > 2 ? 2 : 0)>(i, j, k);
        for (int d = 0; d < D; ++d) {
            int l = slots[d];
            if (l < 0) continue;
            CHECK(l >= G::LOFF[d] && l < G::LOFF[d] + (d == 0 ? G::LX : d == 1 ? G::LY : G::LZ),
                  "D%d slot %d outside array %d\n", D, l, d);
            CHECK(slot_cell.count(l) == 0, "D%d slot %d written twice\n", D, l);
            slot_cell[l] = std::make_tuple(i, j, k);
        }
        CHECK(h >= 0 || slots[0] >= 0, "core cell without x slot\n");
    }
    // 2) face tasks: slots and the 6-cell stencil along d
    auto faces = [&](auto dtag) {
        constexpr int d = decltype(dtag)::value;
        constexpr int BX = G::template BX<d>(), BY = G::template BY<d>();
        constexpr int FD = d == 0 ? G::FX : (d == 1 ? G::FY : G::FZ);
        constexpr int S = G::LSTRIDE[d];
        for (int t = 0; t < FD; ++t) {
            int fi = t % BX, fj = (t / BX) % BY, fk = t / (BX * BY);
            int slot = G::OFF[d] + t;
            CHECK(slot >= 0 && slot < G::F, "slot\n");
            int p[3] = {fi, fj, fk};
            p[d] -= 3;
            int base = G::template lidx<d>(p[0], p[1], p[2]);
            for (int o = 0; o < 6; ++o) {
                int l = base + o * S;
                CHECK(l >= 0 && l < G::L, "D%d dir %d face %d stencil slot %d\n", D, d, t, l);
                auto it = slot_cell.find(l);
                CHECK(it != slot_cell.end(), "D%d dir %d face %d reads unstaged slot %d\n", D, d, t, l);
                if (it == slot_cell.end()) continue;
                int want[3] = {fi, fj, fk};
                want[d] += o - 3;
                CHECK(std::get<0>(it->second) == want[0] && std::get<1>(it->second) == want[1] &&
                          std::get<2>(it->second) == want[2],
                      "D%d dir %d face %d stencil %d reads the wrong cell\n", D, d, t, o);
            }
        }
    };
    faces(std::integral_constant<int, 0>{});
    if (D > 1) faces(std::integral_constant<int, (D > 1 ? 1 : 0)>{});
    if (D > 2) faces(std::integral_constant<int, (D > 2 ? 2 : 0)>{});
    // 3) owned cells: lo/hi face slots decode to the cell's faces; own slot holds the cell
    for (int tid = 0; tid < G::T; ++tid) {
        int li = tid % G::TX, lj = (tid / G::TX) % G::TY, lk = tid / (G::TX * G::TY);
        int flo[3], fhi[3];
        flo[0] = G::OFF[0] + li + (G::TX + 1) * (lj + G::TY * lk);
        fhi[0] = flo[0] + 1;
        flo[1] = D > 1 ? G::OFF[1] + li + G::TX * (lj + (G::TY + 1) * lk) : 0;
        fhi[1] = flo[1] + G::TX;
        flo[2] = D > 2 ? G::OFF[2] + li + G::TX * (lj + G::TY * lk) : 0;
        fhi[2] = flo[2] + G::TX * G::TY;
        for (int d = 0; d < D; ++d) {
            CHECK(flo[d] >= G::OFF[d] && fhi[d] < G::F, "own face slot\n");
            int bx = G::TX + (d == 0), by = G::TY + (d == 1);
            int tl = flo[d] - G::OFF[d], th = fhi[d] - G::OFF[d];
            int cl[3] = {tl % bx, (tl / bx) % by, tl / (bx * by)};
            int ch[3] = {th % bx, (th / bx) % by, th / (bx * by)};
            int me[3] = {li, lj, lk};
            for (int e = 0; e < 3; ++e) {
                CHECK(cl[e] == me[e], "lo face coord\n");
                CHECK(ch[e] == me[e] + (e == d), "hi face coord\n");
            }
        }
        int ol = G::template lidx<0>(li, lj, lk);
        auto it = slot_cell.find(ol);
        CHECK(it != slot_cell.end() && it->second == std::make_tuple(li, lj, lk), "own slot\n");
    }
}

template <int D, int TX, int TY, int TZ>
void check_grid(int nx, int ny, int nz, int bc)
{
    using G = Geo<D, TX, TY, TZ>;
    int n[3] = {nx, D > 1 ? ny : 1, D > 2 ? nz : 1};
    long long N = (long long)n[0] * n[1] * n[2];
    int nt[3] = {(n[0] + G::TX - 1) / G::TX, (n[1] + G::TY - 1) / G::TY, (n[2] + G::TZ - 1) / G::TZ};
    int ntiles = nt[0] * nt[1] * nt[2];
    int per = (ntiles + 7) / 8;
    std::set<int> tiles;
    for (int b = 0; b < 8 * per; ++b) {
        int tile = (b & 7) * per + (b >> 3);
        if (tile >= ntiles) continue;
        tiles.insert(tile);
        int tx = tile % nt[0], ty = (tile / nt[0]) % nt[1], tz = tile / (nt[0] * nt[1]);
        int org[3] = {tx * G::TX, ty * G::TY, tz * G::TZ};
        for (int ci = 0; ci < G::C; ++ci) {
            int i, j, k;
            G::cdecode(ci, i, j, k);
            bool f = false;
            int gx = map_coord(org[0] + i, n[0], bc, f);
            int gy = D > 1 ? map_coord(org[1] + j, n[1], bc, f) : 0;
            int gz = D > 2 ? map_coord(org[2] + k, n[2], bc, f) : 0;
            long long gi = gx + (long long)n[0] * (gy + (long long)n[1] * gz);
            CHECK(gi >= 0 && gi < N, "cross global index %lld of %lld\n", gi, N);
        }
        // core pass: 6-cell lines along each direction, transverse coords inside the tile
        for (int d = 0; d < D; ++d)
            for (int t = 0; t < G::T; ++t) {
                int lc[3] = {t % G::TX, (t / G::TX) % G::TY, t / (G::TX * G::TY)};
                for (int f = 0; f <= (d == 0 ? G::TX : d == 1 ? G::TY : G::TZ); ++f)
                    for (int o = 0; o < 6; ++o) {
                        int cc[3];
                        bool fl = false;
                        for (int e = 0; e < 3; ++e)
                            cc[e] = e < D ? map_coord(org[e] + (e == d ? f - 3 + o : lc[e]), n[e], bc, fl) : 0;
                        long long gi = cc[0] + (long long)n[0] * (cc[1] + (long long)n[1] * cc[2]);
                        CHECK(gi >= 0 && gi < N, "core global index\n");
                    }
            }
    }
    CHECK((int)tiles.size() == ntiles, "tile cover %zu of %d\n", tiles.size(), ntiles);
}

template <int TX>
void check_1d()
{
    check_tile<1, TX, 1, 1>();
    for (int bc = 0; bc < 2; ++bc)
        for (int nx : {bc ? 3 : 1, 5, TX, TX + 1, 400, 1000}) check_grid<1, TX, 1, 1>(nx, 1, 1, bc);
}

template <int TX, int TY>
void check_2d()
{
    check_tile<2, TX, TY, 1>();
    for (int bc = 0; bc < 2; ++bc) {
        int lo = bc ? 3 : 1;
        for (int nx : {lo, 7, TX, TX + 1, 70})
            for (int ny : {lo + 1, TY, TY + 1, 37}) check_grid<2, TX, TY, 1>(nx, ny, 1, bc);
    }
}

template <int TX, int TY, int TZ>
void check_3d()
{
    check_tile<3, TX, TY, TZ>();
    for (int bc = 0; bc < 2; ++bc) {
        int lo = bc ? 3 : 1;
        for (int nx : {lo, TX, 20})
            for (int ny : {lo, TY + 1})
                for (int nz : {lo + 1, TZ, 11}) check_grid<3, TX, TY, TZ>(nx, ny, nz, bc);
    }
}

int main()
{
    // every tile shape the library instantiates
    check_1d<255>();
    check_1d<127>();
    check_1d<511>();
    check_2d<32, 8>();
    check_2d<31, 8>();
    check_2d<64, 4>();
    check_2d<32, 16>();
    check_2d<32, 15>();
    check_2d<16, 15>();
    check_3d<8, 8, 4>();
    check_3d<16, 4, 4>();
    check_3d<8, 4, 4>();
    check_3d<8, 8, 3>();
    check_3d<8, 8, 7>();
    std::printf("%s (%d failures)\n", failures ? "FAIL" : "OK", failures);
    return failures ? 1 : 0;
}
