// Grouped launches of a batch of resident problems (gfx950).
//
// One launch runs one phase of an RK3 step (primitive pass, time step, bubble
// half-step or RK stage) for every member of a launch list.  Its blocks are the
// members' blocks laid end to end: a block finds its member by a binary search
// over the list's prefix offsets and then runs exactly the block body of the
// single-problem kernel on that member's buffers, so every member's result is
// bitwise the one it gets alone.  The member table and the lists live in device
// memory owned by the batch; the host fills them in pinned staging buffers and
// uploads them on the batch's stream ahead of the launches that read them.
#pragma once

#include "device_common.hpp"
#include "ee_kernels.hpp"
#include "split_kernels.hpp"
#include "stage_kernel.hpp"

namespace bub {

constexpr int BATCH_MAX = 256;   // members of one batch

// One member, as the grouped kernels see it.
struct BatchMember {
    double *q, *w1, *w2;          // state and the two stage results
    double *P;                    // primitive scratch
    Scalars *sc;                  // time step, error word, wave-speed maxima
    Grid g;
    Phys ph;
    Bins bt;
    double cfl;
    double rtol;                  // split-mode sub-step tolerance and attempt budget
    int max_substeps;
    int sources;                  // 1: bubble sources inside the stages (unsplit mode)
    // stage decomposition for the member's tile shape (as the single-problem launch computes it)
    int ntile[3], ntiles, ngroups, bpg, nitems;
};

// The members of one launch: member[j] owns blocks (or stage items) start[j] .. start[j+1]-1.
struct LaunchList {
    int count;
    int start[BATCH_MAX + 1];
    int member[BATCH_MAX];
};

// Index j of the list entry that owns block b (0 <= b < start[count]).
__host__ __device__ inline int list_find(const LaunchList *L, int b)
{
    int lo = 0, hi = L->count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L->start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Which of a member's three states a phase reads or writes.
__device__ __forceinline__ double *member_state(const BatchMember &m, int which)
{
    return which == 0 ? m.q : (which == 1 ? m.w1 : m.w2);
}

template <int D, int MODE, int S, int CELLS>
__global__ void __launch_bounds__(S * CELLS) k_prim_group(const BatchMember *__restrict__ tab,
                                                          const LaunchList *__restrict__ L, int which)
{
    __shared__ double s_pp[PPOW_N];
    if (threadIdx.x < PPOW_N) s_pp[threadIdx.x] = PPOW_TABLE[threadIdx.x];
    __syncthreads();
    const int j = list_find(L, blockIdx.x);
    const BatchMember &m = tab[L->member[j]];
    prim_block<D, MODE, S, CELLS, CT_FIFTHS>(member_state(m, which), m.P, m.g, m.ph, m.bt, m.sc, blockIdx.x - L->start[j], s_pp);
}

// The step of every listed member from its wave-speed maxima: one block of WMAX_SLOTS threads each.
__global__ void __launch_bounds__(WMAX_SLOTS) k_dt_group(const BatchMember *__restrict__ tab,
                                                         const LaunchList *__restrict__ L)
{
    const BatchMember &m = tab[L->member[blockIdx.x]];
    dt_block(m.sc, 0.0, m.cfl, nullptr);
}

// Bubble half-step over half the member's own step.
template <int D, int S, int CELLS>
__global__ void __launch_bounds__(S * CELLS) k_bubble_group(const BatchMember *__restrict__ tab,
                                                            const LaunchList *__restrict__ L)
{
    const int j = list_find(L, blockIdx.x);
    const BatchMember &m = tab[L->member[j]];
    BubbleArgs A{};
    A.q = m.q;
    A.taup = &m.sc->dt;
    A.tau_scale = 0.5;
    A.rtol = m.rtol;
    A.max_substeps = m.max_substeps;
    bubble_block<D, S, CELLS, CT_FIFTHS>(A, m.g, m.ph, m.bt, m.sc, blockIdx.x - L->start[j]);
}

// RK stage k (1, 2 or 3) of every listed member; list offsets count stage items.  Blocks are mapped
// to items XCD-aware over the whole launch, so a member's consecutive items share an XCD.
template <int D, int TX_, int TY_, int TZ_, int BLOCK, typename TF>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu((D <= 2 && sizeof(TF) == 4) ? 5 : 1))) k_stage_group(const BatchMember *__restrict__ tab, const LaunchList *__restrict__ L, int stage, int nblk_per_xcd)
{
    BUB_STAGE_SHARED(D, TX_, TY_, TZ_, BLOCK, TF, 2)
    const int b = blockIdx.x;
    const int item = (b & 7) * nblk_per_xcd + (b >> 3);
    if (item >= L->start[L->count]) return;
    const int j = list_find(L, item);
    const BatchMember &m = tab[L->member[j]];
    StageArgs A{};
    A.P = m.P;
    A.dtp = &m.sc->dt;
    A.sources = m.sources;
    A.sc = m.sc;
    A.ntile[0] = m.ntile[0];
    A.ntile[1] = m.ntile[1];
    A.ntile[2] = m.ntile[2];
    A.ntiles = m.ntiles;
    A.ngroups = m.ngroups;
    A.bpg = m.bpg;
    A.nitems = m.nitems;
    if (stage == 1) {
        A.qk = m.q; A.qn = nullptr; A.qo = m.w1; A.a = 0.0; A.b = 1.0;
    } else if (stage == 2) {
        A.qk = m.w1; A.qn = m.q; A.qo = m.w2; A.a = 0.75; A.b = 0.25;
    } else {
        A.qk = m.w2; A.qn = m.q; A.qo = m.q; A.a = 1.0 / 3.0; A.b = 2.0 / 3.0;
    }
    stage_item<D, TX_, TY_, TZ_, BLOCK, TF, false, CT_FIFTHS>(A, m.g, m.ph, m.bt, item - L->start[j], s_coef, s_scr, s_flag,
                                                   s_out, s_pp);
}

// Completion flags in host memory: flags[slot] = epoch once the work queued before this kernel is done.
__global__ void k_flag_set(int *flags, int slot, int epoch)
{
    if (threadIdx.x == 0) {
        __threadfence_system();
        __hip_atomic_store(&flags[slot], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace bub
