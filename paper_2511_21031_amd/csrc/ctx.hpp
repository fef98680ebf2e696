// Context of one problem: host copies of the inputs, the bin table, and the
// context-owned device buffers (bin table, primitive scratch, scalars).
#pragma once

#include <vector>

#include "bubbly.h"
#include "device_common.hpp"

// One timed launch: events recorded on the launch stream around the kernel.
struct ProfRec {
    hipEvent_t a = nullptr, b = nullptr;
    int kind = 0;
};

struct bub_ctx {
    int device = 0;
    bub_grid grid{};
    bub_liquid liq{};
    bub_gas gas{};
    bub_bins bins{};
    bub_opts opts{};
    int ndim = 0, nb = 0, nvar = 0, nprim = 0;
    long long N = 0;
    double h_r0[bub::NB_MAX]{}, h_w[bub::NB_MAX]{}, h_pg0[bub::NB_MAX]{};
    double h_pb0[bub::NB_MAX]{}, h_mv0[bub::NB_MAX]{}, h_mg[bub::NB_MAX]{};   // transfer contents
    double *d_bins = nullptr;    // [BIN_FIELDS][nb]: r0, w, pg0, pb0, mv0, mg
    double *d_P = nullptr;       // [nprim][N] primitive scratch
    double *d_P2 = nullptr;      // second primitive scratch of the fused stages (grids of 2^19 cells or more)
    bub::Scalars *d_sc = nullptr;
    bub::Phys ph{};
    bub::Grid g{};
    bub::Bins bt{};
    bool owns = true;            // device buffers allocated (and freed) by the library
    int tile = 0;                // stage-kernel tile shape (index into the per-dimension list)
    int bin_groups = 0;          // stage-kernel workgroups per tile (0: chosen per launch from the tile count)
    int32_t *nsub_diag = nullptr;   // split-mode steps record their sub-step counts here ([2][nb][N])
    bool src_on = false;         // one-way acoustic source set (bub_set_source)
    bub_source src{};
    int prof_on = 0;
    size_t prof_used = 0;
    std::vector<ProfRec> prof;
};
