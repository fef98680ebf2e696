// Launch lists of a batch's grouped launches (host code, shared with the host-side index check).
//
// Members are grouped by kernel class: the primitive pass and the bubble half-step by
// (dimensionality, threads per cell), the stage by (dimensionality, tile shape), the time step
// over all members.  Each group becomes one LaunchList whose prefix offsets lay the members'
// blocks (or stage items) end to end in slot order.
#pragma once

#include <cstdint>
#include <vector>

#include "batch_kernels.hpp"

namespace bub {

struct PlanMember {
    int slot;              // batch slot (index into the member table)
    int ndim;
    int slots_per_cell;    // threads per cell of the primitive pass and bubble half-step
    int tile;              // stage tile shape index
    bool split;            // bubble half-steps (split mode)
    long long pblocks;     // primitive/bubble blocks
    long long nitems;      // stage work items (tiles x bin groups)
};

struct PlanLaunch {
    int d, key, list;      // key: threads per cell (prim/bubble) or tile shape (stage)
    long long blocks;
};

struct BatchPlan {
    std::vector<LaunchList> lists;
    std::vector<PlanLaunch> prim_all, prim_split, stage;
    int dt_list = -1, dt_count = 0;
};

// 0 on success; -1 if the members need more than max_lists lists or a launch exceeds 2^31 blocks.
inline int plan_batch(const std::vector<PlanMember> &members, int max_lists, BatchPlan *p)
{
    *p = BatchPlan{};
    auto add_to = [&](std::vector<PlanLaunch> &v, int d, int key, int slot, long long blocks) -> int {
        size_t k = 0;
        while (k < v.size() && !(v[k].d == d && v[k].key == key)) ++k;
        if (k == v.size()) {
            if ((int)p->lists.size() >= max_lists) return -1;
            v.push_back({d, key, (int)p->lists.size(), 0});
            p->lists.emplace_back();
            p->lists.back().count = 0;
            p->lists.back().start[0] = 0;
        }
        LaunchList &L = p->lists[v[k].list];
        if (L.count >= BATCH_MAX || blocks < 1 || v[k].blocks + blocks > (long long)INT32_MAX) return -1;
        L.member[L.count] = slot;
        L.start[L.count + 1] = L.start[L.count] + (int)blocks;
        ++L.count;
        v[k].blocks += blocks;
        return 0;
    };
    std::vector<PlanLaunch> dt;
    for (const PlanMember &m : members) {
        if (add_to(p->prim_all, m.ndim, m.slots_per_cell, m.slot, m.pblocks)) return -1;
        if (m.split && add_to(p->prim_split, m.ndim, m.slots_per_cell, m.slot, m.pblocks)) return -1;
        if (add_to(p->stage, m.ndim, m.tile, m.slot, m.nitems)) return -1;
        if (add_to(dt, 0, 0, m.slot, 1)) return -1;
    }
    if (!dt.empty()) {
        p->dt_list = dt[0].list;
        p->dt_count = p->lists[dt[0].list].count;
    }
    return 0;
}

}  // namespace bub
