// Host-side check of the grouped batch launches' block -> (member, block or item) decode (no GPU use).
//
// For many random member sets (dimensionality, threads per cell, tile shape, split mode, block and
// item counts), build the launch lists exactly as the library does (plan_batch), then enumerate every
// block of every grouped launch the way its kernel decodes it: the primitive and bubble launches by
// list_find on the block index, the stage launches through the XCD-aware item order, the time-step
// launch by the list entry.  Exit status 0 only if every block lands on a listed member, inside that
// member's own range, and every (member, block or item) is visited exactly once.
#include <cstdio>
#include <map>
#include <random>
#include <set>
#include <utility>

#include "batch_plan.hpp"

using namespace bub;

static int failures = 0;
#define CHECK(cond, ...)                                 \
    do {                                                 \
        if (!(cond)) {                                   \
            if (failures < 20) std::printf(__VA_ARGS__); \
            ++failures;                                  \
        }                                                \
    } while (0)

static void check_list(const LaunchList &L, const std::map<int, long long> &want, bool stage)
{
    const long long total = L.start[L.count];
    long long sum = 0;
    for (auto &kv : want) sum += kv.second;
    CHECK(total == sum, "list total %lld != %lld\n", total, sum);
    CHECK(L.count == (int)want.size(), "list count\n");
    for (int j = 0; j < L.count; ++j) {
        CHECK(want.count(L.member[j]) == 1, "member %d not planned\n", L.member[j]);
        CHECK(L.start[j + 1] - L.start[j] == want.at(L.member[j]), "member %d range\n", L.member[j]);
    }
    std::map<int, std::set<long long>> seen;
    auto visit = [&](int blk) {
        const int j = list_find(&L, blk);
        CHECK(j >= 0 && j < L.count, "block %d -> entry %d\n", blk, j);
        if (j < 0 || j >= L.count) return;
        const long long local = blk - L.start[j];
        const int m = L.member[j];
        CHECK(local >= 0 && local < want.at(m), "block %d -> member %d local %lld of %lld\n", blk, m, local,
              want.at(m));
        CHECK(seen[m].insert(local).second, "member %d local %lld twice\n", m, local);
    };
    if (!stage) {
        for (long long b = 0; b < total; ++b) visit((int)b);
    } else {
        const int per_xcd = (int)((total + 7) / 8);
        for (int b = 0; b < 8 * per_xcd; ++b) {
            const int item = (b & 7) * per_xcd + (b >> 3);
            if (item >= total) continue;
            visit(item);
        }
    }
    for (auto &kv : want) CHECK((long long)seen[kv.first].size() == kv.second, "member %d coverage\n", kv.first);
}

int main()
{
    std::mt19937 rng(2511);
    const int slots_opts[4] = {1, 2, 4, 8};
    const int tiles_per_dim[4] = {0, 3, 6, 5};
    for (int trial = 0; trial < 400; ++trial) {
        const int max_cases = 1 + (int)(rng() % (trial < 200 ? 16 : BATCH_MAX));
        std::vector<PlanMember> pm;
        for (int slot = 0; slot < max_cases; ++slot) {
            if (rng() % 3 == 0) continue;   // free slot
            PlanMember m;
            m.slot = slot;
            m.ndim = 1 + (int)(rng() % 3);
            m.slots_per_cell = slots_opts[rng() % 4];
            m.tile = (int)(rng() % tiles_per_dim[m.ndim]);
            m.split = rng() % 2;
            m.pblocks = 1 + (long long)(rng() % (trial % 7 == 0 ? 20000 : 300));
            m.nitems = 1 + (long long)(rng() % (trial % 5 == 0 ? 9000 : 400));
            pm.push_back(m);
        }
        BatchPlan p;
        if (plan_batch(pm, 48, &p)) {
            CHECK(false, "plan failed (%zu members)\n", pm.size());
            continue;
        }
        std::map<std::pair<int, int>, std::map<int, long long>> prim, split, stage;
        std::map<int, long long> dt;
        for (auto &m : pm) {
            prim[{m.ndim, m.slots_per_cell}][m.slot] = m.pblocks;
            if (m.split) split[{m.ndim, m.slots_per_cell}][m.slot] = m.pblocks;
            stage[{m.ndim, m.tile}][m.slot] = m.nitems;
            dt[m.slot] = 1;
        }
        CHECK(p.prim_all.size() == prim.size() && p.prim_split.size() == split.size() && p.stage.size() == stage.size(),
              "group counts\n");
        for (auto &l : p.prim_all) check_list(p.lists[l.list], prim[{l.d, l.key}], false);
        for (auto &l : p.prim_split) check_list(p.lists[l.list], split[{l.d, l.key}], false);
        for (auto &l : p.stage) check_list(p.lists[l.list], stage[{l.d, l.key}], true);
        if (!pm.empty()) {
            CHECK(p.dt_list >= 0 && p.dt_count == (int)pm.size(), "dt list\n");
            if (p.dt_list >= 0) check_list(p.lists[p.dt_list], dt, false);
        } else {
            CHECK(p.dt_list == -1 && p.lists.empty(), "empty batch\n");
        }
        for (auto &l : p.prim_all) CHECK(l.blocks == p.lists[l.list].start[p.lists[l.list].count], "launch blocks\n");
        for (auto &l : p.stage) CHECK(l.blocks == p.lists[l.list].start[p.lists[l.list].count], "launch items\n");
    }
    std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
    return failures ? 1 : 0;
}
