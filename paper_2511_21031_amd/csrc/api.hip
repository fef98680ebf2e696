// C ABI of libbubbly.so (declared in include/bubbly.h): contexts, argument
// checks, and the launch sequences of the ensemble-averaged hot path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>

#include "bubbly.h"
#include "ee_kernels.hpp"
#include "split_kernels.hpp"
#include "stage_kernel.hpp"
#include "el_kernels.hpp"
#include "batch_kernels.hpp"
#include "batch_plan.hpp"
#include "viscous_kernel.hpp"
#include "source_kernel.hpp"

#include <vector>
#include "ctx.hpp"

using namespace bub;

#define HIP_OK(expr)                                   \
    do {                                               \
        if ((expr) != hipSuccess) return BUB_EHIP;     \
    } while (0)

namespace {

constexpr size_t PROF_MAX = 65536;

// Returns the record index to close with prof_end, or -1 when not timing.
long prof_begin(bub_ctx *c, int kind, hipStream_t s)
{
    if (!c->prof_on || c->prof_used >= PROF_MAX) return -1;
    if (c->prof_used == c->prof.size()) {
        ProfRec r;
        // timing only: no system-scope release at the end event, whose cache write-back would
        // otherwise be counted into the kernel's time
        if (hipEventCreateWithFlags(&r.a, hipEventDisableSystemFence) != hipSuccess ||
            hipEventCreateWithFlags(&r.b, hipEventDisableSystemFence) != hipSuccess)
            return -1;
        c->prof.push_back(r);
    }
    ProfRec &r = c->prof[c->prof_used];
    r.kind = kind;
    if (hipEventRecord(r.a, s) != hipSuccess) return -1;
    return (long)c->prof_used++;
}

void prof_end(bub_ctx *c, long idx, hipStream_t s)
{
    if (idx >= 0) (void)hipEventRecord(c->prof[idx].b, s);
}

// Host bin table: ln(R0/R_med) on [-3 sigma, 3 sigma], composite Simpson
// weights of the normal pdf, normalised (Sec. 2.2: log-normal bins, Simpson's rule).
int make_bins(int nb, double rmed, double sig, double *r0, double *w)
{
    if (nb < 1 || nb > NB_MAX || nb % 2 == 0 || !(rmed > 0.0)) return BUB_EINVAL;
    if (nb == 1) {
        r0[0] = rmed;
        w[0] = 1.0;
        return BUB_OK;
    }
    if (!(sig > 0.0)) return BUB_EINVAL;
    const double h = 6.0 * sig / (nb - 1);
    const double norm = 1.0 / (sig * std::sqrt(2.0 * M_PI));
    double total = 0.0;
    for (int i = 0; i < nb; ++i) {
        double x = -3.0 * sig + i * h;
        double coef = (i == 0 || i == nb - 1) ? 1.0 : (i & 1 ? 4.0 : 2.0);
        r0[i] = rmed * std::exp(x);
        w[i] = coef * (h / 3.0) * norm * std::exp(-0.5 * x * x / (sig * sig));
        total += w[i];
    }
    for (int i = 0; i < nb; ++i) w[i] /= total;
    return BUB_OK;
}

int blocks_for(long long n, int per = 256)
{
    long long b = (n + per - 1) / per;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (int)b;
}

// Tile shapes of the stage kernel per dimensionality: (TX, TY, TZ, BLOCK).
// Shape 0 is the default; the autotuner may pick another per context.
template <int D, int V> struct Tile;
template <> struct Tile<1, 0> { static constexpr int TX = 255, TY = 1, TZ = 1, BLOCK = 256; };
template <> struct Tile<1, 1> { static constexpr int TX = 127, TY = 1, TZ = 1, BLOCK = 128; };
template <> struct Tile<1, 2> { static constexpr int TX = 511, TY = 1, TZ = 1, BLOCK = 512; };
template <> struct Tile<2, 0> { static constexpr int TX = 32, TY = 8, TZ = 1, BLOCK = 256; };
template <> struct Tile<2, 1> { static constexpr int TX = 31, TY = 8, TZ = 1, BLOCK = 256; };
template <> struct Tile<2, 2> { static constexpr int TX = 64, TY = 4, TZ = 1, BLOCK = 256; };
template <> struct Tile<2, 3> { static constexpr int TX = 32, TY = 16, TZ = 1, BLOCK = 512; };
template <> struct Tile<3, 0> { static constexpr int TX = 8, TY = 8, TZ = 4, BLOCK = 256; };
template <> struct Tile<3, 1> { static constexpr int TX = 16, TY = 4, TZ = 4, BLOCK = 256; };
template <> struct Tile<3, 2> { static constexpr int TX = 8, TY = 4, TZ = 4, BLOCK = 128; };
// Balanced shapes: at most one face per thread in every direction ((TX+1) TY TZ <= BLOCK, ...),
// so no wave carries extra face work into the barrier that follows the face phase.
template <> struct Tile<2, 4> { static constexpr int TX = 32, TY = 15, TZ = 1, BLOCK = 512; };
template <> struct Tile<2, 5> { static constexpr int TX = 16, TY = 15, TZ = 1, BLOCK = 256; };
template <> struct Tile<3, 3> { static constexpr int TX = 8, TY = 8, TZ = 3, BLOCK = 256; };
template <> struct Tile<3, 4> { static constexpr int TX = 8, TY = 8, TZ = 7, BLOCK = 512; };
constexpr int TILE_COUNT[4] = {0, 3, 6, 5};

template <int D, int V>
void tile_info(int *tx, int *ty, int *tz, int *block)
{
    *tx = Tile<D, V>::TX;
    *ty = Tile<D, V>::TY;
    *tz = Tile<D, V>::TZ;
    *block = Tile<D, V>::BLOCK;
}

// The kernels are compiled for the bubble contents (Contents): polytropic gas whose power x^(3 kappa)
// takes the fifth-root Newton form when 3 kappa is a whole number of fifths (air's 4.2, 3, 5, ...) or the
// general exp2(3 kappa log2 x) form otherwise, or transfer contents.  Only the fifth-root form has every
// stage shape; the others run stage shape 0, transfer contents with the fused epilogue where it applies,
// the general power with the separate primitive pass.
int ct_of(const bub_ctx *c)
{
    if (c->opts.contents == BUB_CONTENTS_TRANSFER) return CT_TRANSFER;
    return c->ph.pw_c > 0 ? CT_FIFTHS : CT_POLY;
}
bool pw_fast(const bub_ctx *c) { return ct_of(c) == CT_FIFTHS; }

template <int D, int S, int CELLS, int CT>
void launch_prim_p(bub_ctx *c, const double *q, double *out, int mode, hipStream_t s)
{
    const dim3 grid((unsigned)((c->g.N + CELLS - 1) / CELLS)), block(S * CELLS);
    if (mode == PRIM_CFL)
        hipLaunchKernelGGL((k_prim<D, PRIM_CFL, S, CELLS, CT>), grid, block, 0, s, q, out, c->g, c->ph, c->bt,
                           c->d_sc);
    else if (mode == PRIM_MOMENTS)
        hipLaunchKernelGGL((k_prim<D, PRIM_MOMENTS, S, CELLS, CT>), grid, block, 0, s, q, out, c->g, c->ph, c->bt,
                           c->d_sc);
    else
        hipLaunchKernelGGL((k_prim<D, PRIM_ONLY, S, CELLS, CT>), grid, block, 0, s, q, out, c->g, c->ph, c->bt,
                           c->d_sc);
}

template <int D, int S, int CELLS>
void launch_prim_s(bub_ctx *c, const double *q, double *out, int mode, hipStream_t s)
{
    switch (ct_of(c)) {
    case CT_FIFTHS: launch_prim_p<D, S, CELLS, CT_FIFTHS>(c, q, out, mode, s); break;
    case CT_TRANSFER: launch_prim_p<D, S, CELLS, CT_TRANSFER>(c, q, out, mode, s); break;
    default: launch_prim_p<D, S, CELLS, CT_POLY>(c, q, out, mode, s); break;
    }
}

template <int D>
int launch_prim(bub_ctx *c, const double *q, double *out, int mode, hipStream_t s)
{
    long pr = prof_begin(c, BUB_K_PRIM, s);
    switch (slots_for(c->g.N)) {
    case 1: launch_prim_s<D, 1, 256>(c, q, out, mode, s); break;
    case 2: launch_prim_s<D, 2, 64>(c, q, out, mode, s); break;
    case 4: launch_prim_s<D, 4, 64>(c, q, out, mode, s); break;
    default: launch_prim_s<D, 8, 64>(c, q, out, mode, s); break;
    }
    prof_end(c, pr, s);
    return hipGetLastError() == hipSuccess ? BUB_OK : BUB_EHIP;
}

// Bin groups: small grids give each tile several workgroups (a range of bins each) so the launch
// still fills the chip; large grids keep one workgroup per tile (no repeated mixture faces).
// Returns the bins per group; *groups receives the workgroups per tile.
int bin_grouping(const bub_ctx *c, long long ntiles, int *groups)
{
    int ng = c->bin_groups;
    if (ng <= 0) {
        constexpr int target = 1024;   // work items that keep 256 CUs busy
        ng = ntiles >= target ? 1 : (int)((target + ntiles - 1) / ntiles);
        const int cap = (c->nb + 1) / 2;  // at least two bins per group
        if (ng > cap) ng = cap;
    }
    if (ng < 1) ng = 1;
    if (ng > c->nb) ng = c->nb;
    const int bpg = (c->nb + ng - 1) / ng;
    *groups = (c->nb + bpg - 1) / bpg;
    return bpg;
}

template <int D, int V, typename TF>
int launch_stage_t(bub_ctx *c, StageArgs A, hipStream_t s)
{
    using TC = Tile<D, V>;
    using G = Geo<D, TC::TX, TC::TY, TC::TZ>;
    A.ntile[0] = (c->g.n[0] + G::TX - 1) / G::TX;
    A.ntile[1] = (c->g.n[1] + G::TY - 1) / G::TY;
    A.ntile[2] = (c->g.n[2] + G::TZ - 1) / G::TZ;
    A.ntiles = A.ntile[0] * A.ntile[1] * A.ntile[2];
    A.bpg = bin_grouping(c, A.ntiles, &A.ngroups);
    if (A.Pout && A.ngroups != 1) return BUB_EINVAL;   // the fused epilogue needs every bin of a cell
    A.nitems = A.ntiles * A.ngroups;
    A.nblk_per_xcd = (A.nitems + 7) / 8;
    const dim3 grid(8 * A.nblk_per_xcd), block(TC::BLOCK);
    if (!pw_fast(c)) {
        if constexpr (V == 0) {
            const bool tr = ct_of(c) == CT_TRANSFER;
            if (A.Pout && !tr) return BUB_EINVAL;   // (stage_fusable is false for the general power)
            long pr = prof_begin(c, BUB_K_STAGE, s);
            if (tr && A.Pout)
                hipLaunchKernelGGL((k_stage<D, TC::TX, TC::TY, TC::TZ, TC::BLOCK, TF, true, CT_TRANSFER>), grid,
                                   block, 0, s, A, c->g, c->ph, c->bt);
            else if (tr)
                hipLaunchKernelGGL((k_stage<D, TC::TX, TC::TY, TC::TZ, TC::BLOCK, TF, false, CT_TRANSFER>), grid,
                                   block, 0, s, A, c->g, c->ph, c->bt);
            else
                hipLaunchKernelGGL((k_stage<D, TC::TX, TC::TY, TC::TZ, TC::BLOCK, TF, false, CT_POLY>), grid, block,
                                   0, s, A, c->g, c->ph, c->bt);
            prof_end(c, pr, s);
            return hipGetLastError() == hipSuccess ? BUB_OK : BUB_EHIP;
        }
        return BUB_EUNSUPPORTED;
    }
    long pr = prof_begin(c, BUB_K_STAGE, s);
    if (A.Pout)
        hipLaunchKernelGGL((k_stage<D, TC::TX, TC::TY, TC::TZ, TC::BLOCK, TF, true, CT_FIFTHS>), grid, block, 0, s,
                           A, c->g, c->ph, c->bt);
    else
        hipLaunchKernelGGL((k_stage<D, TC::TX, TC::TY, TC::TZ, TC::BLOCK, TF, false, CT_FIFTHS>), grid, block, 0, s,
                           A, c->g, c->ph, c->bt);
    prof_end(c, pr, s);
    return hipGetLastError() == hipSuccess ? BUB_OK : BUB_EHIP;
}

template <int D, int V>
int launch_stage_v(bub_ctx *c, StageArgs A, hipStream_t s)
{
    if (c->opts.precision == BUB_PREC_MIXED) return launch_stage_t<D, V, float>(c, A, s);
    return launch_stage_t<D, V, double>(c, A, s);
}

template <int D, int S, int CELLS>
void launch_bubble_s(bub_ctx *c, const BubbleArgs &B, hipStream_t s)
{
    const dim3 grid((unsigned)((c->g.N + CELLS - 1) / CELLS)), block(S * CELLS);
    switch (ct_of(c)) {
    case CT_FIFTHS:
        hipLaunchKernelGGL((k_bubble<D, S, CELLS, CT_FIFTHS>), grid, block, 0, s, B, c->g, c->ph, c->bt, c->d_sc);
        break;
    case CT_TRANSFER:
        hipLaunchKernelGGL((k_bubble<D, S, CELLS, CT_TRANSFER>), grid, block, 0, s, B, c->g, c->ph, c->bt, c->d_sc);
        break;
    default:
        hipLaunchKernelGGL((k_bubble<D, S, CELLS, CT_POLY>), grid, block, 0, s, B, c->g, c->ph, c->bt, c->d_sc);
        break;
    }
}

template <int D>
void launch_bubble_d(bub_ctx *c, const BubbleArgs &B, hipStream_t s)
{
    switch (slots_for(c->g.N)) {
    case 1: launch_bubble_s<D, 1, 256>(c, B, s); break;
    case 2: launch_bubble_s<D, 2, 64>(c, B, s); break;
    case 4: launch_bubble_s<D, 4, 64>(c, B, s); break;
    default: launch_bubble_s<D, 8, 64>(c, B, s); break;
    }
}

int bubble(bub_ctx *c, double *q, const double *taup, double tau_scale, double tau_fixed, int *nsub,
           hipStream_t s)
{
    BubbleArgs B{};
    B.q = q;
    B.taup = taup;
    B.tau_scale = tau_scale;
    B.tau_fixed = tau_fixed;
    B.rtol = c->opts.sub_rtol > 0.0 ? c->opts.sub_rtol : 1e-4;
    B.max_substeps = c->opts.max_substeps > 0 ? c->opts.max_substeps : 10000;
    B.nsub = nsub;
    long pr = prof_begin(c, BUB_K_OTHER, s);
    switch (c->ndim) {
    case 1: launch_bubble_d<1>(c, B, s); break;
    case 2: launch_bubble_d<2>(c, B, s); break;
    default: launch_bubble_d<3>(c, B, s); break;
    }
    prof_end(c, pr, s);
    return hipGetLastError() == hipSuccess ? BUB_OK : BUB_EHIP;
}

int prim(bub_ctx *c, const double *q, double *out, int mode, hipStream_t s)
{
    switch (c->ndim) {
    case 1: return launch_prim<1>(c, q, out, mode, s);
    case 2: return launch_prim<2>(c, q, out, mode, s);
    default: return launch_prim<3>(c, q, out, mode, s);
    }
}

int stage_kernel(bub_ctx *c, const StageArgs &A, hipStream_t s)
{
    const int v = pw_fast(c) ? c->tile : 0;
    switch (c->ndim) {
    case 1:
        if (v == 1) return launch_stage_v<1, 1>(c, A, s);
        if (v == 2) return launch_stage_v<1, 2>(c, A, s);
        return launch_stage_v<1, 0>(c, A, s);
    case 2:
        if (v == 1) return launch_stage_v<2, 1>(c, A, s);
        if (v == 2) return launch_stage_v<2, 2>(c, A, s);
        if (v == 3) return launch_stage_v<2, 3>(c, A, s);
        if (v == 4) return launch_stage_v<2, 4>(c, A, s);
        if (v == 5) return launch_stage_v<2, 5>(c, A, s);
        return launch_stage_v<2, 0>(c, A, s);
    default:
        if (v == 1) return launch_stage_v<3, 1>(c, A, s);
        if (v == 2) return launch_stage_v<3, 2>(c, A, s);
        if (v == 3) return launch_stage_v<3, 3>(c, A, s);
        if (v == 4) return launch_stage_v<3, 4>(c, A, s);
        return launch_stage_v<3, 0>(c, A, s);
    }
}

// The source pass: the launch description of the context's source (cells that can lie within 6
// widths of the plane); false when no cell can.
bool source_launch(const bub_ctx *c, Source *S)
{
    const bub_source &q = c->src;
    const int d = q.dir;
    const double dx = c->grid.dx[d];
    const int n = c->g.n[d];
    long long lo = (long long)std::floor((q.x - 6.0 * q.width) / dx - 0.5) - 1;
    long long hi = (long long)std::ceil((q.x + 6.0 * q.width) / dx - 0.5) + 1;
    if (lo < 0) lo = 0;
    if (hi > n - 1) hi = n - 1;
    if (hi < lo) return false;
    const double c0 = std::sqrt(c->liq.gamma * (c->liq.p0 + c->liq.pi_inf) / c->liq.rho0);
    const double k = 2.0 * M_PI * q.freq / c0;
    *S = Source{};
    S->dir = d;
    S->sign = q.sign;
    S->lo = (int)lo;
    for (int e = 0; e < 3; ++e) S->m[e] = e == d ? (int)(hi - lo + 1) : c->g.n[e];
    S->x = q.x;
    S->width = q.width;
    S->dx = dx;
    S->norm = 1.0 / (std::sqrt(2.0 * M_PI) * q.width);
    S->amp_eff = q.amp * std::exp(0.5 * (k * q.width) * (k * q.width));
    S->omega = 2.0 * M_PI * q.freq;
    S->t0 = q.t0;
    S->dur = q.ncycles > 0.0 ? q.ncycles / q.freq : 0.0;
    S->c0 = c0;
    S->inv_c0 = 1.0 / c0;
    S->inv_gm1 = 1.0 / (c->liq.gamma - 1.0);
    return true;
}

// An RK stage (or a right-hand side): the stage kernel, then the passes that add what the stage kernels
// carry no code for: the stress of eq. stressTensor (viscous problems) and the acoustic source.  tc: the
// stage's time within the step (0, 1, 1/2 for stages 1, 2, 3; negative for a right-hand side).
int stage(bub_ctx *c, const StageArgs &A, hipStream_t s, double tc)
{
    int rc = stage_kernel(c, A, s);
    if (rc) return rc;
    if (c->opts.viscous && c->gas.mu > 0.0) {
        long pr = prof_begin(c, BUB_K_OTHER, s);
        const dim3 grid(blocks_for(c->N)), block(256);
        const double *dtp = A.rhs_mode ? nullptr : A.dtp;
        switch (c->ndim) {
        case 1: hipLaunchKernelGGL((k_viscous<1>), grid, block, 0, s, A.P, A.qo, c->g, c->gas.mu, dtp, A.b); break;
        case 2: hipLaunchKernelGGL((k_viscous<2>), grid, block, 0, s, A.P, A.qo, c->g, c->gas.mu, dtp, A.b); break;
        default: hipLaunchKernelGGL((k_viscous<3>), grid, block, 0, s, A.P, A.qo, c->g, c->gas.mu, dtp, A.b); break;
        }
        prof_end(c, pr, s);
        HIP_OK(hipGetLastError());
    }
    Source S;
    if (c->src_on && source_launch(c, &S)) {
        long pr = prof_begin(c, BUB_K_OTHER, s);
        const long long cells = (long long)S.m[0] * S.m[1] * S.m[2];
        const dim3 grid((unsigned)std::min<long long>((cells + 255) / 256, 2048)), block(256);
        const double t = A.rhs_mode ? -1.0 : tc;
        switch (c->ndim) {
        case 1: hipLaunchKernelGGL((k_source<1>), grid, block, 0, s, A.P, A.qo, c->g, S, c->d_sc, t, A.b); break;
        case 2: hipLaunchKernelGGL((k_source<2>), grid, block, 0, s, A.P, A.qo, c->g, S, c->d_sc, t, A.b); break;
        default: hipLaunchKernelGGL((k_source<3>), grid, block, 0, s, A.P, A.qo, c->g, S, c->d_sc, t, A.b); break;
        }
        prof_end(c, pr, s);
        HIP_OK(hipGetLastError());
    }
    return BUB_OK;
}

// Tiles of the context's current stage shape.
long long stage_tiles(const bub_ctx *c)
{
    int tx, ty, tz, blk;
    bub_tile_info(c, c->tile, &tx, &ty, &tz, &blk);
    return (long long)((c->g.n[0] + tx - 1) / tx) * ((c->g.n[1] + ty - 1) / ty) * ((c->g.n[2] + tz - 1) / tz);
}

// The stage kernels can carry the primitive pass of the state they write (fused epilogue) when one
// workgroup owns all bins of a tile and the grid is large enough that the primitive pass would take
// one thread per cell (then both forms sum the bins in the same order, so results are bitwise equal).
bool stage_fusable(const bub_ctx *c)
{
    // (a viscous or source pass after the stage changes the state the epilogue would describe)
    if (!c->d_P2 || slots_for(c->N) != 1 || c->opts.viscous || c->src_on || ct_of(c) == CT_POLY) return false;
    // 3D FP64: the epilogue's registers cost the stage more than the pass it saves (measured at 256^3
    // x 21 bins: 13.6 ms fused against 11.9 + 1.5 ms)
    if (c->ndim == 3 && c->opts.precision == BUB_PREC_FP64) return false;
    int groups = 0;
    bin_grouping(c, stage_tiles(c), &groups);
    return groups == 1;
}

}  // namespace

extern "C" {

const char *bub_strerror(int code)
{
    switch (code) {
    case BUB_OK: return "ok";
    case BUB_EINVAL: return "invalid argument";
    case BUB_ENOMEM: return "out of memory";
    case BUB_EHIP: return "HIP runtime error";
    case BUB_ENONFINITE: return "non-finite or inadmissible state";
    case BUB_ENEGR: return "non-positive bubble radius";
    case BUB_ESUBSTEP: return "bubble sub-step budget exhausted";
    case BUB_EUNSUPPORTED: return "unsupported request";
    default: return "unknown error";
    }
}

}  // extern "C"

namespace {

// Bin table passed by value to the initialising kernel (no host memory to keep alive): BIN_FIELDS
// arrays of nb values (r0, w, pg0, and the transfer contents' pb0, mv0, mg).
constexpr int BIN_FIELDS = 6;
struct BinTable {
    double v[BIN_FIELDS * NB_MAX];
};

__global__ void k_ctx_init(double *bins, BinTable t, int n, Scalars *sc)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) bins[i] = t.v[i];
    for (int i = threadIdx.x; i < WMAX_SLOTS * WMAX_STRIDE; i += blockDim.x) sc->wmax[i] = 0ull;
    if (threadIdx.x == 0) {
        sc->dt = 0.0;
        sc->err_code = 0;
        sc->err_bin = 0;
        sc->err_cell = 0;
        sc->t = 0.0;
        sc->t_next = 0.0;
    }
}

__global__ void k_set_time(Scalars *sc, double t)
{
    if (threadIdx.x == 0) {
        sc->t = t;
        sc->t_next = t;
    }
}

__global__ void k_err_copy(const Scalars *sc, int64_t *dst)
{
    if (threadIdx.x == 0) {
        const int code = sc->err_code;
        dst[0] = code;
        dst[1] = code ? (int64_t)sc->err_cell : -1;
        dst[2] = code ? (int64_t)sc->err_bin : -1;
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device-buffer layout of a context: bin table | scalars | primitive scratch | second primitive
// scratch (only for grids of 2^19 cells or more, whose stages carry the primitive pass; off_P2 = 0
// otherwise).
void ctx_buffer_layout(int ndim, long long N, size_t *off_sc, size_t *off_P, size_t *off_P2, size_t *total)
{
    const size_t pbytes = align256(sizeof(double) * (size_t)(ndim + 6) * (size_t)N);
    *off_sc = align256(sizeof(double) * BIN_FIELDS * NB_MAX);
    *off_P = *off_sc + align256(sizeof(Scalars));
    *off_P2 = slots_for(N) == 1 ? *off_P + pbytes : 0;
    *total = *off_P + pbytes + (*off_P2 ? pbytes : 0);
}

void ctx_finish(bub_ctx *c)
{
    c->bt.r0 = c->d_bins;
    c->bt.w = c->d_bins + c->nb;
    c->bt.pg0 = c->d_bins + 2 * c->nb;
    c->bt.pb0 = c->d_bins + 3 * c->nb;
    c->bt.mv0 = c->d_bins + 4 * c->nb;
    c->bt.mg = c->d_bins + 5 * c->nb;
}

void bin_table(const bub_ctx *c, double *tab)
{
    const double *f[BIN_FIELDS] = {c->h_r0, c->h_w, c->h_pg0, c->h_pb0, c->h_mv0, c->h_mg};
    for (int k = 0; k < BIN_FIELDS; ++k) std::memcpy(tab + k * c->nb, f[k], sizeof(double) * c->nb);
}

// Validate the inputs and fill the host side of a context held by the caller (no allocation).
int ctx_fill(const bub_grid *grid, const bub_liquid *liq, const bub_gas *gas, const bub_bins *bins,
             const bub_opts *opts, bub_ctx *c)
{
    if (!grid || !liq || !gas || !bins || !opts || !c) return BUB_EINVAL;
    if (grid->ndim < 1 || grid->ndim > 3) return BUB_EINVAL;
    long long N = 1;
    for (int d = 0; d < 3; ++d) {
        if (grid->n[d] < 1) return BUB_EINVAL;
        if (d >= grid->ndim && grid->n[d] != 1) return BUB_EINVAL;
        if (d < grid->ndim) {
            if (!(grid->dx[d] > 0.0)) return BUB_EINVAL;
            int lo = grid->bc[d][0], hi = grid->bc[d][1];
            if (lo < 0 || lo > 2 || lo != hi) return BUB_EINVAL;
            if (lo == 1 && grid->n[d] < 3) return BUB_EINVAL;
        }
        N *= grid->n[d];
    }
    if (N >= (1LL << 32)) return BUB_EINVAL;
    if (!(liq->gamma > 1.0) || !(liq->pi_inf >= 0.0) || !(liq->rho0 > 0.0) || !(liq->p0 > 0.0)) return BUB_EINVAL;
    if (!(gas->kappa > 0.0) || !(gas->sigma >= 0.0) || !(gas->mu >= 0.0) || !(gas->pv >= 0.0)) return BUB_EINVAL;
    if (!(opts->cfl > 0.0) || opts->cfl > 1.0) return BUB_EINVAL;
    if (opts->precision != BUB_PREC_FP64 && opts->precision != BUB_PREC_MIXED) return BUB_EINVAL;
    if (opts->bubble_mode != BUB_BUBBLES_UNSPLIT && opts->bubble_mode != BUB_BUBBLES_SPLIT) return BUB_EINVAL;
    if (opts->bubble_mode == BUB_BUBBLES_SPLIT && (!(opts->sub_rtol > 0.0) || opts->max_substeps < 1))
        return BUB_EINVAL;
    if (opts->viscous != 0 && opts->viscous != 1) return BUB_EINVAL;
    if (opts->contents != BUB_CONTENTS_POLYTROPIC && opts->contents != BUB_CONTENTS_TRANSFER) return BUB_EINVAL;
    const bool tr = opts->contents == BUB_CONTENTS_TRANSFER;
    if (tr) {
        const bub_transfer &t = opts->transfer;
        if (!(t.gam_b > 1.0) || !(t.Rg > 0.0) || !(t.Rv > 0.0) || !(t.T0 > 0.0) || !(t.k_b >= 0.0) ||
            !(t.D_v >= 0.0) || !(t.beta_T >= 0.0) || !(t.beta_c >= 0.0) || !(gas->pv < liq->p0))
            return BUB_EINVAL;
    }

    c->grid = *grid;
    c->liq = *liq;
    c->gas = *gas;
    c->bins = *bins;
    c->opts = *opts;
    int rc = make_bins(bins->nb, bins->r0_median, bins->sigma_ln, c->h_r0, c->h_w);
    if (rc) return rc;
    c->ndim = grid->ndim;
    c->nb = bins->nb;
    const int nf = tr ? 4 : 2;
    c->nvar = c->ndim + 3 + nf * c->nb;
    c->nprim = c->ndim + 6;
    c->N = N;
    double m3 = 0.0;
    const bub_transfer &t = opts->transfer;
    for (int i = 0; i < c->nb; ++i) {
        c->h_pg0[i] = liq->p0 + 2.0 * gas->sigma / c->h_r0[i] - gas->pv;
        m3 += c->h_w[i] * c->h_r0[i] * c->h_r0[i] * c->h_r0[i];
        c->h_pb0[i] = c->h_mv0[i] = c->h_mg[i] = 0.0;
        if (tr) {
            // equilibrium: contents at the Laplace pressure, vapour saturated at T0, the rest gas at T0
            const double V0 = FOUR_PI_3 * c->h_r0[i] * c->h_r0[i] * c->h_r0[i];
            c->h_pb0[i] = liq->p0 + 2.0 * gas->sigma / c->h_r0[i];
            c->h_mv0[i] = gas->pv * V0 / (t.Rv * t.T0);
            c->h_mg[i] = (c->h_pb0[i] - gas->pv) * V0 / (t.Rg * t.T0);
        }
    }
    if (hipGetDevice(&c->device) != hipSuccess) return BUB_EHIP;
    c->ph.gamma = liq->gamma;
    c->ph.pi_inf = liq->pi_inf;
    c->ph.gm1 = liq->gamma - 1.0;
    c->ph.inv_gm1 = 1.0 / (liq->gamma - 1.0);
    c->ph.gpi = liq->gamma * liq->pi_inf;
    c->ph.kappa3 = 3.0 * gas->kappa;
    c->ph.sigma2 = 2.0 * gas->sigma;
    c->ph.mu4 = 4.0 * gas->mu;
    c->ph.p0 = liq->p0;
    c->ph.rho0 = liq->rho0;
    if (tr) {
        c->ph.g3 = 3.0 * t.gam_b;
        c->ph.Rg = t.Rg;
        c->ph.Rv = t.Rv;
        c->ph.T0 = t.T0;
        c->ph.pv = gas->pv;
        c->ph.kh = (t.gam_b - 1.0) / t.gam_b * t.k_b;
        c->ph.betaT = t.beta_T;
        c->ph.dbc = t.D_v * t.beta_c;
        c->ph.pvRg = gas->pv * t.Rg;
        c->ph.RvT0 = t.Rv * t.T0;
        c->ph.inv_RgRv2T0 = 1.0 / (t.Rg * t.Rv * t.Rv * t.T0);
    }
    // 3 kappa = n / 5 for a whole n (kappa = 1, 1.4, 5/3, ...): the fifth-root power
    const double n5 = 5.0 * c->ph.kappa3;
    const long long n = std::llround(n5);
    c->ph.pw_c = c->ph.pw_d = 0;
    if (n >= 1 && n <= 100 && std::fabs(n5 - (double)n) <= 1e-12 * (double)n) {
        c->ph.pw_c = (int)((n + 4) / 5);
        c->ph.pw_d = (int)(5 * c->ph.pw_c - n);
    }
    for (int d = 0; d < 3; ++d) {
        c->g.n[d] = grid->n[d];
        c->g.bc[d] = d < grid->ndim ? grid->bc[d][0] : 0;
        c->g.inv_dx[d] = d < grid->ndim ? 1.0 / grid->dx[d] : 0.0;
    }
    c->g.N = N;
    ctx_finish(c);
    c->bt.nb = c->nb;
    c->bt.nf = nf;
    c->bt.m3_eq = m3;
    return BUB_OK;
}

// Validate the inputs and build the host side of a heap context (no device memory yet).
int ctx_setup(const bub_grid *grid, const bub_liquid *liq, const bub_gas *gas, const bub_bins *bins,
              const bub_opts *opts, bub_ctx **out)
{
    if (!out) return BUB_EINVAL;
    *out = nullptr;
    bub_ctx *c = new (std::nothrow) bub_ctx();
    if (!c) return BUB_ENOMEM;
    const int rc = ctx_fill(grid, liq, gas, bins, opts, c);
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return BUB_OK;
}

}  // namespace

extern "C" {

int bub_ctx_create(const bub_grid *grid, const bub_liquid *liq, const bub_gas *gas, const bub_bins *bins,
                   const bub_opts *opts, bub_ctx **out)
{
    bub_ctx *c = nullptr;
    int rc = ctx_setup(grid, liq, gas, bins, opts, &c);
    if (rc) return rc;
    size_t pbytes = sizeof(double) * (size_t)c->nprim * (size_t)c->N;
    c->owns = true;
    if (hipMalloc(&c->d_bins, sizeof(double) * BIN_FIELDS * NB_MAX) != hipSuccess ||
        hipMalloc(&c->d_P, pbytes) != hipSuccess || hipMalloc(&c->d_sc, sizeof(Scalars)) != hipSuccess ||
        (slots_for(c->N) == 1 && hipMalloc(&c->d_P2, pbytes) != hipSuccess)) {
        bub_ctx_destroy(c);
        return BUB_ENOMEM;
    }
    double tab[BIN_FIELDS * NB_MAX];
    bin_table(c, tab);
    Scalars zero{};
    if (hipMemcpy(c->d_bins, tab, sizeof(double) * BIN_FIELDS * c->nb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_sc, &zero, sizeof(Scalars), hipMemcpyHostToDevice) != hipSuccess) {
        bub_ctx_destroy(c);
        return BUB_EHIP;
    }
    ctx_finish(c);
    *out = c;
    return BUB_OK;
}

int bub_ctx_buffer_bytes(const bub_grid *grid, const bub_bins *bins, size_t *bytes)
{
    if (!grid || !bins || !bytes || grid->ndim < 1 || grid->ndim > 3) return BUB_EINVAL;
    long long N = 1;
    for (int d = 0; d < 3; ++d) {
        if (grid->n[d] < 1) return BUB_EINVAL;
        N *= grid->n[d];
    }
    size_t a, b, p2;
    ctx_buffer_layout(grid->ndim, N, &a, &b, &p2, bytes);
    return BUB_OK;
}

int bub_ctx_create_on(const bub_grid *grid, const bub_liquid *liq, const bub_gas *gas, const bub_bins *bins,
                      const bub_opts *opts, void *buffer, size_t bytes, void *stream, bub_ctx **out)
{
    if (!buffer || ((uintptr_t)buffer & 255)) return BUB_EINVAL;
    bub_ctx *c = nullptr;
    int rc = ctx_setup(grid, liq, gas, bins, opts, &c);
    if (rc) return rc;
    size_t off_sc, off_P, off_P2, total;
    ctx_buffer_layout(c->ndim, c->N, &off_sc, &off_P, &off_P2, &total);
    if (bytes < total) {
        delete c;
        return BUB_EINVAL;
    }
    char *base = (char *)buffer;
    c->owns = false;
    c->d_bins = (double *)base;
    c->d_sc = (Scalars *)(base + off_sc);
    c->d_P = (double *)(base + off_P);
    c->d_P2 = off_P2 ? (double *)(base + off_P2) : nullptr;
    BinTable t{};
    bin_table(c, t.v);
    hipLaunchKernelGGL(k_ctx_init, dim3(1), dim3(64), 0, (hipStream_t)stream, c->d_bins, t, BIN_FIELDS * c->nb, c->d_sc);
    if (hipGetLastError() != hipSuccess) {
        delete c;
        return BUB_EHIP;
    }
    ctx_finish(c);
    *out = c;
    return BUB_OK;
}

int bub_ctx_destroy(bub_ctx *c)
{
    if (!c) return BUB_EINVAL;
    if (c->owns) {
        (void)hipDeviceSynchronize();
        if (c->d_bins) (void)hipFree(c->d_bins);
        if (c->d_P) (void)hipFree(c->d_P);
        if (c->d_P2) (void)hipFree(c->d_P2);
        if (c->d_sc) (void)hipFree(c->d_sc);
    }
    for (ProfRec &r : c->prof) {
        if (r.a) (void)hipEventDestroy(r.a);
        if (r.b) (void)hipEventDestroy(r.b);
    }
    delete c;
    return BUB_OK;
}

int bub_layout(const bub_ctx *c, int *nvar, int *nprim, int64_t *ncells, size_t *state_bytes, size_t *work_bytes)
{
    if (!c) return BUB_EINVAL;
    size_t sb = sizeof(double) * (size_t)c->nvar * (size_t)c->N;
    if (nvar) *nvar = c->nvar;
    if (nprim) *nprim = c->nprim;
    if (ncells) *ncells = c->N;
    if (state_bytes) *state_bytes = sb;
    if (work_bytes) *work_bytes = 2 * sb;
    return BUB_OK;
}

int bub_bins_get(const bub_ctx *c, double *r0, double *w)
{
    if (!c || !r0 || !w) return BUB_EINVAL;
    std::memcpy(r0, c->h_r0, sizeof(double) * c->nb);
    std::memcpy(w, c->h_w, sizeof(double) * c->nb);
    return BUB_OK;
}

int bub_init_state(bub_ctx *c, const double *prim_in, double *q, void *stream)
{
    if (!c || !prim_in || !q) return BUB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int nbk = blocks_for(c->N);
    switch (c->ndim) {
    case 1: hipLaunchKernelGGL((k_init<1>), dim3(nbk), dim3(256), 0, s, prim_in, q, c->g, c->ph, c->bt); break;
    case 2: hipLaunchKernelGGL((k_init<2>), dim3(nbk), dim3(256), 0, s, prim_in, q, c->g, c->ph, c->bt); break;
    default: hipLaunchKernelGGL((k_init<3>), dim3(nbk), dim3(256), 0, s, prim_in, q, c->g, c->ph, c->bt); break;
    }
    return hipGetLastError() == hipSuccess ? BUB_OK : BUB_EHIP;
}

int bub_moments(bub_ctx *c, const double *q, double *out, void *stream)
{
    if (!c || !q || !out || q == out) return BUB_EINVAL;
    return prim(c, q, out, PRIM_MOMENTS, (hipStream_t)stream);
}

}  // extern "C"

namespace {

int rhs_stage_impl(bub_ctx *c, const double *q, double *rhs, hipStream_t s)
{
    int rc = prim(c, q, c->d_P, PRIM_ONLY, s);
    if (rc) return rc;
    StageArgs A{};
    A.qk = q;
    A.qn = nullptr;
    A.qo = rhs;
    A.P = c->d_P;
    A.dtp = nullptr;
    A.a = 0.0;
    A.b = 1.0;
    A.rhs_mode = 1;
    A.sources = c->opts.bubble_mode == BUB_BUBBLES_UNSPLIT;
    return stage(c, A, s, -1.0);
}

}  // namespace

extern "C" {

int bub_rhs_stage(bub_ctx *c, const double *q, double *rhs, void *stream)
{
    if (!c || !q || !rhs || q == rhs) return BUB_EINVAL;
    return rhs_stage_impl(c, q, rhs, (hipStream_t)stream);
}

}  // extern "C"

namespace {

// nsteps SSP-RK3 steps (Sec. 3).  With the fused epilogue (stage_fusable), stages 1 and 2 write the
// primitives of the state they produce (P -> P2 -> P), so only the step's first stage needs a
// primitive pass; in unsplit mode stage 3 of every step but the last also writes the primitives and
// the wave-speed maxima of u^{n+1}, so the next step needs none.  Results are bitwise those of the
// unfused sequence (same arithmetic, same bin order).
int rk3_steps_impl(bub_ctx *c, double *q, double *work, int nsteps, double dt, double *dt_dev, hipStream_t s)
{
    const bool split = c->opts.bubble_mode == BUB_BUBBLES_SPLIT;
    const size_t M = (size_t)c->nvar * (size_t)c->N;
    double *w1 = work, *w2 = work + M;
    const bool cfl = !(dt > 0.0);
    const bool fuse = stage_fusable(c);
    const bool carry = fuse && !split;   // the last bubble half-step of split mode changes u^{n+1}
    double *Pa = c->d_P, *Pb = c->d_P2;  // Pa: primitives of the step's starting state
    int rc = BUB_OK;
    for (int k = 0; k < nsteps; ++k) {
        const bool more = k + 1 < nsteps;
        if ((k == 0 || !carry) && (rc = prim(c, q, Pa, cfl ? PRIM_CFL : PRIM_ONLY, s))) return rc;
        long pr = prof_begin(c, BUB_K_OTHER, s);
        hipLaunchKernelGGL(k_dt, dim3(1), dim3(WMAX_SLOTS), 0, s, c->d_sc, cfl ? 0.0 : dt, c->opts.cfl, dt_dev);
        prof_end(c, pr, s);
        HIP_OK(hipGetLastError());
        if (split) {
            // S_b(dt/2) first; the flux part then starts from the primitives of the advanced state
            if ((rc = bubble(c, q, &c->d_sc->dt, 0.5, 0.0, c->nsub_diag, s))) return rc;
            if ((rc = prim(c, q, Pa, PRIM_ONLY, s))) return rc;
        }
        StageArgs A{};
        A.dtp = &c->d_sc->dt;
        A.rhs_mode = 0;
        A.sources = split ? 0 : 1;
        A.sc = c->d_sc;
        // stage 1: u1 = u^n + dt L(u^n)
        A.qk = q; A.qn = nullptr; A.qo = w1; A.a = 0.0; A.b = 1.0;
        A.P = Pa;
        A.Pout = fuse ? Pb : nullptr;
        if ((rc = stage(c, A, s, 0.0))) return rc;
        // stage 2: u2 = 3/4 u^n + 1/4 (u1 + dt L(u1))
        if (!fuse && (rc = prim(c, w1, Pa, PRIM_ONLY, s))) return rc;
        A.qk = w1; A.qn = q; A.qo = w2; A.a = 0.75; A.b = 0.25;
        A.P = fuse ? Pb : Pa;
        A.Pout = fuse ? Pa : nullptr;
        if ((rc = stage(c, A, s, 1.0))) return rc;
        // stage 3: u^{n+1} = 1/3 u^n + 2/3 (u2 + dt L(u2)), written over u^n (own-cell reads only)
        if (!fuse && (rc = prim(c, w2, Pa, PRIM_ONLY, s))) return rc;
        A.qk = w2; A.qn = q; A.qo = q; A.a = 1.0 / 3.0; A.b = 2.0 / 3.0;
        A.P = Pa;
        A.Pout = carry && more ? Pb : nullptr;
        A.cfl = carry && more && cfl;
        if ((rc = stage(c, A, s, 0.5))) return rc;
        if (split &&   // S_b(dt/2)
            (rc = bubble(c, q, &c->d_sc->dt, 0.5, 0.0,
                         c->nsub_diag ? c->nsub_diag + (size_t)c->nb * c->N : nullptr, s)))
            return rc;
        if (carry && more) std::swap(Pa, Pb);
    }
    return rc;
}

int rk3_check(const bub_ctx *c, const double *q, const double *work, double dt)
{
    if (!c || !q || !work) return BUB_EINVAL;
    if (!(dt == dt) || dt == INFINITY) return BUB_EINVAL;
    const size_t M = (size_t)c->nvar * (size_t)c->N;
    if ((q >= work && q < work + 2 * M) || (work >= q && work < q + M)) return BUB_EINVAL;
    return BUB_OK;
}

}  // namespace

extern "C" {

int bub_rk3_step(bub_ctx *c, double *q, double *work, double dt, double *dt_dev, void *stream)
{
    int rc = rk3_check(c, q, work, dt);
    return rc ? rc : rk3_steps_impl(c, q, work, 1, dt, dt_dev, (hipStream_t)stream);
}

int bub_rk3_steps(bub_ctx *c, double *q, double *work, int nsteps, double dt, double *dt_dev, void *stream)
{
    int rc = rk3_check(c, q, work, dt);
    if (rc) return rc;
    if (nsteps < 0) return BUB_EINVAL;
    return rk3_steps_impl(c, q, work, nsteps, dt, dt_dev, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Volume-averaged (Euler--Lagrange) variant
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

int el_grid(const bub_ctx *c, ElGrid *g)
{
    if (c->ndim != 3) return BUB_EUNSUPPORTED;
    if (c->opts.contents != BUB_CONTENTS_POLYTROPIC) return BUB_EUNSUPPORTED;   // Lagrangian bubbles: polytropic
    if (c->grid.dx[1] != c->grid.dx[0] || c->grid.dx[2] != c->grid.dx[0]) return BUB_EUNSUPPORTED;
    for (int d = 0; d < 3; ++d) {
        g->n[d] = c->g.n[d];
        g->bc[d] = c->g.bc[d];
        if (g->n[d] < 3 || g->bc[d] > 1) return BUB_EUNSUPPORTED;   // periodic or reflective only
    }
    g->dx = c->grid.dx[0];
    g->inv_dx = 1.0 / g->dx;
    g->N = c->N;
    return BUB_OK;
}

int el_prim(bub_ctx *c, const ElGrid &g, const double *ql, bool cfl, hipStream_t s)
{
    long pr = prof_begin(c, BUB_K_PRIM, s);
    if (cfl)
        hipLaunchKernelGGL((k_el_prim<true>), dim3(blocks_for(g.N)), dim3(256), 0, s, ql, c->d_P, g, c->ph, c->d_sc);
    else
        hipLaunchKernelGGL((k_el_prim<false>), dim3(blocks_for(g.N)), dim3(256), 0, s, ql, c->d_P, g, c->ph, c->d_sc);
    prof_end(c, pr, s);
    return hipGetLastError() == hipSuccess ? BUB_OK : BUB_EHIP;
}

int el_smear(bub_ctx *c, const ElGrid &g, const double *b, long long nb, double *aD, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(2 * g.N)), dim3(256), 0, s, aD, 2 * g.N, 0.0);
    if (nb > 0) {
        long pr = prof_begin(c, BUB_K_OTHER, s);
        hipLaunchKernelGGL(k_el_scatter, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, s, b, nb, g, aD);
        prof_end(c, pr, s);
    }
    return hipGetLastError() == hipSuccess ? BUB_OK : BUB_EHIP;
}

// gather from the liquid primitives P, then advance every bubble over (*taup) * scale
int el_bubbles(bub_ctx *c, const ElGrid &g, const double *P, double *b, long long nb, double *forcing,
               const double *taup, double scale, int *nsub, hipStream_t s)
{
    if (nb <= 0) return BUB_OK;
    long pr = prof_begin(c, BUB_K_OTHER, s);
    hipLaunchKernelGGL(k_el_gather, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, s, P, b, nb, g, c->ph, forcing);
    ElOdeArgs O{};
    O.b = b;
    O.nb = nb;
    O.forcing = forcing;
    O.taup = taup;
    O.tau_scale = scale;
    O.rtol = c->opts.sub_rtol > 0.0 ? c->opts.sub_rtol : 1e-4;
    O.max_substeps = c->opts.max_substeps > 0 ? c->opts.max_substeps : 10000;
    O.nsub = nsub;
    if (pw_fast(c)) hipLaunchKernelGGL(k_el_ode<true>, dim3(blocks_for(nb)), dim3(256), 0, s, O, c->ph, c->d_sc);
    else hipLaunchKernelGGL(k_el_ode<false>, dim3(blocks_for(nb)), dim3(256), 0, s, O, c->ph, c->d_sc);
    prof_end(c, pr, s);
    return hipGetLastError() == hipSuccess ? BUB_OK : BUB_EHIP;
}

int el_stage(bub_ctx *c, const ElGrid &g, ElStageArgs A, hipStream_t s)
{
    long pr = prof_begin(c, BUB_K_STAGE, s);
    const int ntx = (g.n[0] + ELT_X - 1) / ELT_X, nty = (g.n[1] + ELT_Y - 1) / ELT_Y;
    const int ntz = (g.n[2] + ELT_Z - 1) / ELT_Z;
    const int ntiles = ntx * nty * ntz, per_xcd = (ntiles + 7) / 8;
    hipLaunchKernelGGL(k_el_stage, dim3(8u * (unsigned)per_xcd), dim3(ELT_BLOCK), 0, s, A, g, c->ph, ntx, nty, ntiles,
                       per_xcd);
    prof_end(c, pr, s);
    return hipGetLastError() == hipSuccess ? BUB_OK : BUB_EHIP;
}

__global__ void k_fill_i(int *p, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace

extern "C" {

int bub_lagrangian_layout(const bub_ctx *c, int64_t nbub, size_t *work_bytes)
{
    ElGrid g;
    if (!c || !work_bytes || nbub < 0) return BUB_EINVAL;
    int rc = el_grid(c, &g);
    if (rc) return rc;
    *work_bytes = sizeof(double) * (size_t)(15 * g.N + 3 * nbub);
    return BUB_OK;
}

int bub_lagrangian_bubbles(bub_ctx *c, const double *xyzr0, double *bubbles, int64_t nbub, void *stream)
{
    ElGrid g;
    if (!c || nbub < 0 || (nbub > 0 && (!xyzr0 || !bubbles))) return BUB_EINVAL;
    int rc = el_grid(c, &g);
    if (rc || nbub == 0) return rc;
    hipLaunchKernelGGL(k_el_bubinit, dim3(blocks_for(nbub)), dim3(256), 0, (hipStream_t)stream, xyzr0, bubbles,
                       (long long)nbub, c->ph, 2.0 * c->gas.sigma, c->gas.pv);
    return hipGetLastError() == hipSuccess ? BUB_OK : BUB_EHIP;
}

int bub_lagrangian_init(bub_ctx *c, const double *prim_in, double *ql, void *stream)
{
    ElGrid g;
    if (!c || !prim_in || !ql) return BUB_EINVAL;
    int rc = el_grid(c, &g);
    if (rc) return rc;
    hipLaunchKernelGGL(k_el_init, dim3(blocks_for(g.N)), dim3(256), 0, (hipStream_t)stream, prim_in, ql, g.N, c->ph);
    return hipGetLastError() == hipSuccess ? BUB_OK : BUB_EHIP;
}

int bub_lagrangian_smear(bub_ctx *c, const double *bubbles, int64_t nbub, double *alpha_D, void *stream)
{
    ElGrid g;
    if (!c || !alpha_D || nbub < 0 || (nbub > 0 && !bubbles)) return BUB_EINVAL;
    int rc = el_grid(c, &g);
    if (rc) return rc;
    return el_smear(c, g, bubbles, nbub, alpha_D, (hipStream_t)stream);
}

int bub_lagrangian_gather(bub_ctx *c, const double *ql, const double *bubbles, int64_t nbub, double *out,
                          void *stream)
{
    ElGrid g;
    if (!c || !ql || nbub < 0 || (nbub > 0 && (!bubbles || !out))) return BUB_EINVAL;
    int rc = el_grid(c, &g);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = el_prim(c, g, ql, false, s))) return rc;
    if (nbub > 0)
        hipLaunchKernelGGL(k_el_gather, dim3((unsigned)((nbub + 3) / 4)), dim3(256), 0, s, c->d_P, bubbles,
                           (long long)nbub, g, c->ph, out);
    return hipGetLastError() == hipSuccess ? BUB_OK : BUB_EHIP;
}

int bub_lagrangian_rhs(bub_ctx *c, const double *ql, const double *alpha_D, double *rhs, void *stream)
{
    ElGrid g;
    if (!c || !ql || !alpha_D || !rhs || ql == rhs) return BUB_EINVAL;
    int rc = el_grid(c, &g);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = el_prim(c, g, ql, false, s))) return rc;
    ElStageArgs A{};
    A.qk = ql;
    A.qo = rhs;
    A.P = c->d_P;
    A.aD = alpha_D;
    A.b = 1.0;
    A.rhs_mode = 1;
    return el_stage(c, g, A, s);
}

int bub_lagrangian_step(bub_ctx *c, double *ql, double *bubbles, int64_t nbub, double *alpha_D, double *work,
                        double dt, double *dt_dev, int32_t *nsub, void *stream)
{
    return bub_lagrangian_steps(c, ql, bubbles, nbub, alpha_D, work, 1, dt, dt_dev, nsub, stream);
}

int bub_lagrangian_steps(bub_ctx *c, double *ql, double *bubbles, int64_t nbub, double *alpha_D, double *work,
                         int nsteps, double dt, double *dt_dev, int32_t *nsub, void *stream)
{
    ElGrid g;
    if (!c || !ql || !alpha_D || !work || nbub < 0 || nsteps < 0 || (nbub > 0 && !bubbles)) return BUB_EINVAL;
    if (!(dt == dt) || dt == INFINITY) return BUB_EINVAL;
    int rc = el_grid(c, &g);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    // work: the two stage results, the bubbles' forcing and a second primitive buffer.  The stages
    // write the primitives of the state they produce into the buffer they do not read (Pc and Po
    // take turns); the last stage of a step that another step follows also posts that state's wave
    // speeds, so the next step starts from Pc without a primitive pass of its own.
    double *w1 = work, *w2 = work + 5 * g.N, *forcing = work + 10 * g.N;
    double *Pc = c->d_P, *Po = forcing + 3 * nbub;
    const bool cfl = !(dt > 0.0);
    const double *dtp = &c->d_sc->dt;
    for (int k = 0; k < nsteps; ++k) {
        if (k == 0 && (rc = el_prim(c, g, ql, cfl, s))) return rc;
        hipLaunchKernelGGL(k_dt, dim3(1), dim3(WMAX_SLOTS), 0, s, c->d_sc, cfl ? 0.0 : dt, c->opts.cfl, dt_dev);
        if (nsub && nbub > 0)
            hipLaunchKernelGGL(k_fill_i, dim3(blocks_for(nbub)), dim3(256), 0, s, nsub, (long long)nbub);
        if ((rc = el_bubbles(c, g, Pc, bubbles, nbub, forcing, dtp, 0.5, nsub, s))) return rc;
        if ((rc = el_smear(c, g, bubbles, nbub, alpha_D, s))) return rc;
        ElStageArgs A{};
        A.aD = alpha_D;
        A.dtp = dtp;
        A.sc = c->d_sc;
        A.qk = ql; A.qn = nullptr; A.qo = w1; A.a = 0.0; A.b = 1.0; A.P = Pc; A.Pout = Po;
        if ((rc = el_stage(c, g, A, s))) return rc;
        A.qk = w1; A.qn = ql; A.qo = w2; A.a = 0.75; A.b = 0.25; A.P = Po; A.Pout = Pc;
        if ((rc = el_stage(c, g, A, s))) return rc;
        A.qk = w2; A.qn = ql; A.qo = ql; A.a = 1.0 / 3.0; A.b = 2.0 / 3.0; A.P = Pc; A.Pout = Po;
        A.cfl = cfl && k + 1 < nsteps;
        if ((rc = el_stage(c, g, A, s))) return rc;
        if ((rc = el_bubbles(c, g, Po, bubbles, nbub, forcing, dtp, 0.5, nsub, s))) return rc;
        // the closing smear of a step is read by nothing before the next step smears again (its bubble
        // half-step gathers the liquid only), so only the last step's is made
        if (k == nsteps - 1 && (rc = el_smear(c, g, bubbles, nbub, alpha_D, s))) return rc;
        std::swap(Pc, Po);
    }
    return BUB_OK;
}

int bub_bubble_advance(bub_ctx *c, double *q, double tau, int32_t *nsub, void *stream)
{
    if (!c || !q || !(tau > 0.0) || tau == INFINITY) return BUB_EINVAL;
    return bubble(c, q, nullptr, 0.0, tau, nsub, (hipStream_t)stream);
}

int bub_last_error(bub_ctx *c, int *code, int64_t *cell, int *bin, void *stream)
{
    if (!c) return BUB_EINVAL;
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    Scalars h{};
    HIP_OK(hipMemcpy(&h, c->d_sc, sizeof(Scalars), hipMemcpyDeviceToHost));
    if (code) *code = h.err_code;
    if (cell) *cell = h.err_code ? h.err_cell : -1;
    if (bin) *bin = h.err_code ? h.err_bin : -1;
    Scalars cleared = h;
    cleared.err_code = 0;
    cleared.err_bin = 0;
    cleared.err_cell = 0;
    HIP_OK(hipMemcpy(c->d_sc, &cleared, sizeof(Scalars), hipMemcpyHostToDevice));
    return BUB_OK;
}

int bub_error_copy(const bub_ctx *c, int64_t *dst, void *stream)
{
    if (!c || !dst) return BUB_EINVAL;
    hipLaunchKernelGGL(k_err_copy, dim3(1), dim3(64), 0, (hipStream_t)stream, c->d_sc, dst);
    HIP_OK(hipGetLastError());
    return BUB_OK;
}

int bub_substep_counts(bub_ctx *c, int32_t *nsub)
{
    if (!c) return BUB_EINVAL;
    c->nsub_diag = nsub;
    return BUB_OK;
}

int bub_set_source(bub_ctx *c, const bub_source *src)
{
    if (!c) return BUB_EINVAL;
    if (!src) {
        c->src_on = false;
        return BUB_OK;
    }
    if (src->dir < 0 || src->dir >= c->ndim || (src->sign != 1 && src->sign != -1)) return BUB_EINVAL;
    if (!(src->width > 0.0) || !(src->freq > 0.0) || !(src->ncycles >= 0.0) || !std::isfinite(src->amp) ||
        !std::isfinite(src->x) || !std::isfinite(src->t0) || src->width == INFINITY || src->freq == INFINITY)
        return BUB_EINVAL;
    c->src = *src;
    c->src_on = true;
    return BUB_OK;
}

int bub_set_time(bub_ctx *c, double t, void *stream)
{
    if (!c || !std::isfinite(t)) return BUB_EINVAL;
    hipLaunchKernelGGL(k_set_time, dim3(1), dim3(64), 0, (hipStream_t)stream, c->d_sc, t);
    HIP_OK(hipGetLastError());
    return BUB_OK;
}

int bub_get_time(bub_ctx *c, double *t)
{
    if (!c || !t) return BUB_EINVAL;
    HIP_OK(hipDeviceSynchronize());
    Scalars h{};
    HIP_OK(hipMemcpy(&h, c->d_sc, sizeof(Scalars), hipMemcpyDeviceToHost));
    *t = h.t_next;
    return BUB_OK;
}

int bub_bin_groups(bub_ctx *c, int groups)
{
    if (!c || groups < 0) return BUB_EINVAL;
    c->bin_groups = groups;
    return BUB_OK;
}

int bub_tile_count(const bub_ctx *c, int *count)
{
    if (!c || !count) return BUB_EINVAL;
    *count = TILE_COUNT[c->ndim];
    return BUB_OK;
}

int bub_tile_info(const bub_ctx *c, int idx, int *tx, int *ty, int *tz, int *block)
{
    if (!c || !tx || !ty || !tz || !block || idx < 0 || idx >= TILE_COUNT[c->ndim]) return BUB_EINVAL;
    switch (c->ndim * 10 + idx) {
    case 10: tile_info<1, 0>(tx, ty, tz, block); break;
    case 11: tile_info<1, 1>(tx, ty, tz, block); break;
    case 12: tile_info<1, 2>(tx, ty, tz, block); break;
    case 20: tile_info<2, 0>(tx, ty, tz, block); break;
    case 21: tile_info<2, 1>(tx, ty, tz, block); break;
    case 22: tile_info<2, 2>(tx, ty, tz, block); break;
    case 23: tile_info<2, 3>(tx, ty, tz, block); break;
    case 24: tile_info<2, 4>(tx, ty, tz, block); break;
    case 25: tile_info<2, 5>(tx, ty, tz, block); break;
    case 30: tile_info<3, 0>(tx, ty, tz, block); break;
    case 31: tile_info<3, 1>(tx, ty, tz, block); break;
    case 32: tile_info<3, 2>(tx, ty, tz, block); break;
    case 33: tile_info<3, 3>(tx, ty, tz, block); break;
    default: tile_info<3, 4>(tx, ty, tz, block); break;
    }
    return BUB_OK;
}

int bub_tile_set(bub_ctx *c, int idx)
{
    if (!c || idx < 0 || idx >= TILE_COUNT[c->ndim]) return BUB_EINVAL;
    if (idx != 0 && !pw_fast(c)) return BUB_EUNSUPPORTED;
    c->tile = idx;
    return BUB_OK;
}

int bub_tile_get(const bub_ctx *c, int *idx)
{
    if (!c || !idx) return BUB_EINVAL;
    *idx = c->tile;
    return BUB_OK;
}

}  // extern "C"

namespace {

// Tile-shape cache: a text file of lines "<arch> <ndim> <nb> <precision> <size class> <tile>", the size
// class being floor(log2 N).  Lines that do not parse, or name another shape count, are ignored; the
// last matching line wins.
struct TuneKey {
    char arch[64];
    int ndim, nb, precision, size_class;
};

int tune_key(const bub_ctx *c, TuneKey *k)
{
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return BUB_EHIP;
    std::memset(k->arch, 0, sizeof(k->arch));
    for (int i = 0; i < (int)sizeof(k->arch) - 1 && prop.gcnArchName[i] && prop.gcnArchName[i] != ':' &&
                    prop.gcnArchName[i] != ' ';
         ++i)
        k->arch[i] = prop.gcnArchName[i];
    k->ndim = c->ndim;
    k->nb = c->nb;
    k->precision = c->opts.precision;
    int sc = 0;
    while ((1LL << (sc + 1)) <= c->N) ++sc;
    k->size_class = sc;
    return BUB_OK;
}

// The cached tile of key k in the file at path, or -1.
int tune_lookup(const char *path, const TuneKey &k, int ntiles)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return -1;
    char line[256];
    int found = -1;
    while (std::fgets(line, sizeof(line), f)) {
        char arch[64];
        int nd, nb, pr, sc, t;
        if (std::sscanf(line, "%63s %d %d %d %d %d", arch, &nd, &nb, &pr, &sc, &t) != 6) continue;
        if (std::strcmp(arch, k.arch) == 0 && nd == k.ndim && nb == k.nb && pr == k.precision &&
            sc == k.size_class && t >= 0 && t < ntiles)
            found = t;
    }
    std::fclose(f);
    return found;
}

int tune_store(const char *path, const TuneKey &k, int tile)
{
    FILE *f = std::fopen(path, "a");   // one short line per append: whole lines even with concurrent writers
    if (!f) return BUB_EINVAL;
    const int ok = std::fprintf(f, "%s %d %d %d %d %d\n", k.arch, k.ndim, k.nb, k.precision, k.size_class, tile) > 0;
    return std::fclose(f) == 0 && ok ? BUB_OK : BUB_EINVAL;
}

}  // namespace

extern "C" {

int bub_autotune_cached(bub_ctx *c, const char *cache_path, const double *q, double *scratch, int reps, int *best,
                        int *hit, void *stream)
{
    if (!c || !cache_path) return BUB_EINVAL;
    if (!pw_fast(c)) {   // one stage shape: nothing to choose or to store
        if (hit) *hit = 0;
        return bub_autotune(c, q, scratch, reps, nullptr, best, stream);
    }
    TuneKey k;
    int rc = tune_key(c, &k);
    if (rc) return rc;
    const int t = tune_lookup(cache_path, k, TILE_COUNT[c->ndim]);
    if (hit) *hit = t >= 0;
    if (t >= 0) {
        c->tile = t;
        if (best) *best = t;
        return BUB_OK;
    }
    int tb = 0;
    if ((rc = bub_autotune(c, q, scratch, reps, nullptr, &tb, stream))) return rc;
    if (best) *best = tb;
    return tune_store(cache_path, k, tb);
}

int bub_autotune(bub_ctx *c, const double *q, double *scratch, int reps, double *ms_out, int *best, void *stream)
{
    if (!c || !q || !scratch || q == scratch || reps < 1) return BUB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = prim(c, q, c->d_P, PRIM_ONLY, s);
    if (rc) return rc;
    StageArgs A{};
    A.qk = q;
    A.qo = scratch;
    A.P = c->d_P;
    A.b = 1.0;
    A.rhs_mode = 1;
    A.sources = c->opts.bubble_mode == BUB_BUBBLES_UNSPLIT;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    HIP_OK(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
    const int keep = c->tile, prof = c->prof_on;
    c->prof_on = 0;
    double best_ms = 1e300;
    int best_v = keep;
    const int nshape = pw_fast(c) ? TILE_COUNT[c->ndim] : 1;
    if (ms_out)
        for (int v = nshape; v < TILE_COUNT[c->ndim]; ++v) ms_out[v] = -1.0;
    for (int v = 0; v < nshape && rc == BUB_OK; ++v) {
        c->tile = v;
        rc = stage_kernel(c, A, s);  // warm-up (code load)
        if (rc) break;
        if (hipEventRecord(e0, s) != hipSuccess) { rc = BUB_EHIP; break; }
        for (int r = 0; r < reps && rc == BUB_OK; ++r) rc = stage_kernel(c, A, s);
        if (rc) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = BUB_EHIP;
            break;
        }
        double per = ms / reps;
        if (ms_out) ms_out[v] = per;
        if (per < best_ms) {
            best_ms = per;
            best_v = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->prof_on = prof;
    c->tile = rc == BUB_OK ? best_v : keep;
    if (best) *best = c->tile;
    return rc;
}

int bub_profile(bub_ctx *c, int enable)
{
    if (!c) return BUB_EINVAL;
    c->prof_on = enable ? 1 : 0;
    return BUB_OK;
}

int bub_profile_read(bub_ctx *c, int kind, double *total_ms, int64_t *launches)
{
    if (!c || kind < BUB_K_STAGE || kind > BUB_K_OTHER) return BUB_EINVAL;
    HIP_OK(hipDeviceSynchronize());
    double tot = 0.0;
    int64_t cnt = 0;
    size_t keep = 0;
    for (size_t i = 0; i < c->prof_used; ++i) {
        ProfRec &r = c->prof[i];
        if (r.kind == kind) {
            float ms = 0.0f;
            HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
            tot += ms;
            ++cnt;
        } else {
            std::swap(c->prof[keep++], r);
        }
    }
    c->prof_used = keep;
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
    return BUB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: resident problems advanced together, fanned out over a few streams
// ---------------------------------------------------------------------------
struct bub_batch {
    struct Member {
        bub_ctx *ctx = nullptr;
        double *q = nullptr, *work = nullptr;
        bool used = false;
        hipGraphExec_t exec = nullptr;   // one captured rk3_step of this member (graph mode)
        int cap_tile = -1, cap_groups = -1;
        size_t bytes = 0;                // device bytes counted against the budget
        int remaining = 0;               // steps still to take in bub_batch_run (0 with open = false: finished)
        bool open = false;               // added with steps = 0: stepped by every run, never finished
        int done_epoch = 0;              // epoch of the flag that marks its last step done (0: none)
        bool reported = false;           // bub_batch_poll has returned it
    };
    // grouped launches (bub_batch_run)
    size_t budget = 0, used_bytes = 0;            // device bytes of the members; budget 0 = none
    BatchMember *d_tab = nullptr;                 // device member table [max_cases]
    LaunchList *d_lists = nullptr;                // device launch lists [NLISTS]
    static constexpr int NLISTS = 48;
    int *h_flags = nullptr, *d_flags = nullptr;   // completion flags in pinned host memory [max_cases]
    // table and list uploads: a ring of pinned staging buffers, each reused only after the event
    // recorded behind its last upload has completed
    static constexpr int NSTAGE = 8;
    char *h_stage[NSTAGE] = {};
    hipEvent_t stage_ev[NSTAGE] = {};
    bool stage_used[NSTAGE] = {};
    int stage_next = 0;
    int epoch = 0;
    bool dirty = true;                            // table or lists out of date
    int version = 0;                              // bumped whenever they are rewritten
    struct Launch { int d, key, list; long long blocks; };   // key: slots (prim/bubble) or tile (stage)
    std::vector<Launch> prim_all, prim_split, stage_l;
    int dt_list = -1, dt_count = 0;
    hipGraphExec_t run_exec = nullptr;            // captured chunk of grouped launches
    hipEvent_t run_ev = nullptr;                  // recorded after every launch of run_exec
    int run_steps = -1, run_version = -1;
    std::vector<std::pair<hipGraphExec_t, hipEvent_t>> run_retired;   // freed once their event completed
    int precision = 0;
    bool graphs = true;                           // replay each member's step as one captured graph
    hipStream_t cap = nullptr;                    // capture stream (never executes work)
    std::vector<hipGraphExec_t> retired;          // graphs of removed members, freed once the lanes are idle
    std::vector<Member> slots;
    static constexpr int NSTREAM = 16;            // internal streams (lanes) created
    int lanes = 4;                                // lanes used: one per hardware queue a process gets by default
    hipStream_t st[NSTREAM] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[NSTREAM] = {};
    std::vector<std::pair<int, int>> tuned_key;   // (ndim, nb) classes with an autotuned tile
    std::vector<int> tuned_tile;
    std::string tune_cache;                       // tile-shape cache file of the class autotuner ("" = none)
};

namespace {

// bub_batch_run takes the grouped launches (further below) only when this is set.  They are switched
// off: on the GPU a batch run through them once returned corrupted member states and once faulted the
// device, while the same launches run block by block on the host reproduce every member bitwise; the
// cause, somewhere in how the uploaded tables meet the launches that read them on the device, is not
// known yet.  Until it is, bub_batch_run steps each member with its own kernels on the batch's lanes
// (as bub_batch_step).
constexpr bool kGroupedLaunches = false;

// Whether p lies in device memory of the current HIP runtime (host memory, pinned or not, does not).
bool is_device_memory(const void *p)
{
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

int batch_class_tile(const bub_batch *b, const bub_ctx *c)
{
    for (size_t i = 0; i < b->tuned_key.size(); ++i)
        if (b->tuned_key[i].first == c->ndim && b->tuned_key[i].second == c->nb) return b->tuned_tile[i];
    return -1;
}

}  // namespace

namespace {

// Capture one rk3_step of member m (its kernels only: no copies, no memsets) into a graph.
int batch_capture(bub_batch *b, bub_batch::Member &m)
{
    hipGraph_t g = nullptr;
    HIP_OK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const int rc = bub_rk3_step(m.ctx, m.q, m.work, 0.0, nullptr, b->cap);
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : BUB_EHIP;
    }
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return BUB_EHIP;
    if (m.exec) b->retired.push_back(m.exec);
    m.exec = x;
    m.cap_tile = m.ctx->tile;
    m.cap_groups = m.ctx->bin_groups;
    return BUB_OK;
}

int batch_free_retired(bub_batch *b)
{
    for (int k = 0; k < bub_batch::NSTREAM; ++k)
        if (b->st[k]) HIP_OK(hipStreamSynchronize(b->st[k]));
    for (hipGraphExec_t x : b->retired) (void)hipGraphExecDestroy(x);
    b->retired.clear();
    return BUB_OK;
}

}  // namespace

extern "C" {

int bub_batch_create(int precision, int max_cases, size_t hbm_budget, bub_batch **out)
{
    if (!out || max_cases < 1 || max_cases > BATCH_MAX || (precision != BUB_PREC_FP64 && precision != BUB_PREC_MIXED))
        return BUB_EINVAL;
    bub_batch *b = new (std::nothrow) bub_batch();
    if (!b) return BUB_ENOMEM;
    b->precision = precision;
    b->budget = hbm_budget;
    b->slots.resize(max_cases);
    if (hipMalloc(&b->d_tab, sizeof(BatchMember) * (size_t)max_cases) != hipSuccess ||
        hipMalloc(&b->d_lists, sizeof(LaunchList) * (size_t)bub_batch::NLISTS) != hipSuccess ||
        hipHostMalloc(&b->h_flags, sizeof(int) * (size_t)max_cases, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        bub_batch_destroy(b);
        return BUB_ENOMEM;
    }
    std::memset(b->h_flags, 0, sizeof(int) * (size_t)max_cases);
    const size_t stage_bytes = sizeof(BatchMember) * (size_t)max_cases + sizeof(LaunchList) * bub_batch::NLISTS;
    for (int k = 0; k < bub_batch::NSTAGE; ++k) {
        if (hipHostMalloc((void **)&b->h_stage[k], stage_bytes, hipHostMallocDefault) != hipSuccess) {
            bub_batch_destroy(b);
            return BUB_ENOMEM;
        }
        if (hipEventCreateWithFlags(&b->stage_ev[k], hipEventDisableTiming) != hipSuccess) {
            bub_batch_destroy(b);
            return BUB_EHIP;
        }
    }
    if (hipHostGetDevicePointer((void **)&b->d_flags, b->h_flags, 0) != hipSuccess) {
        bub_batch_destroy(b);
        return BUB_EHIP;
    }
    bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess &&
              hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; k < bub_batch::NSTREAM && ok; ++k)
        ok = hipStreamCreateWithFlags(&b->st[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        bub_batch_destroy(b);
        return BUB_EHIP;
    }
    *out = b;
    return BUB_OK;
}

int bub_batch_destroy(bub_batch *b)
{
    if (!b) return BUB_EINVAL;
    (void)batch_free_retired(b);
    for (auto &m : b->slots)
        if (m.exec) (void)hipGraphExecDestroy(m.exec);
    for (int k = 0; k < bub_batch::NSTREAM; ++k) {
        if (b->st[k]) (void)hipStreamDestroy(b->st[k]);
        if (b->join[k]) (void)hipEventDestroy(b->join[k]);
    }
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->d_tab || b->d_lists || b->h_flags || b->h_stage[0]) (void)hipDeviceSynchronize();   // work may still use them
    if (b->run_exec) (void)hipGraphExecDestroy(b->run_exec);
    if (b->run_ev) (void)hipEventDestroy(b->run_ev);
    for (auto &r : b->run_retired) {
        (void)hipGraphExecDestroy(r.first);
        (void)hipEventDestroy(r.second);
    }
    if (b->d_tab) (void)hipFree(b->d_tab);
    if (b->d_lists) (void)hipFree(b->d_lists);
    if (b->h_flags) (void)hipHostFree(b->h_flags);
    for (int k = 0; k < bub_batch::NSTAGE; ++k) {
        if (b->h_stage[k]) (void)hipHostFree(b->h_stage[k]);
        if (b->stage_ev[k]) (void)hipEventDestroy(b->stage_ev[k]);
    }
    delete b;
    return BUB_OK;
}

int bub_batch_add(bub_batch *b, bub_ctx *c, double *q, double *work, int steps, int *slot)
{
    if (!b || !c || !q || !work || !slot || steps < 0) return BUB_EINVAL;
    if (c->opts.precision != b->precision) return BUB_EINVAL;
    if (kGroupedLaunches && (c->opts.viscous || c->src_on))
        return BUB_EUNSUPPORTED;   // the grouped launches carry no viscous or source pass
    const size_t M = (size_t)c->nvar * (size_t)c->N;
    if ((q >= work && q < work + 2 * M) || (work >= q && work < q + M)) return BUB_EINVAL;
    for (size_t i = 0; i < b->slots.size(); ++i) {
        auto &m = b->slots[i];
        if (m.used && m.ctx == c) return BUB_EINVAL;
    }
    // every pointer the grouped kernels will read from the member table must be device memory
    if (!is_device_memory(q) || !is_device_memory(work) || !is_device_memory(c->d_P) ||
        !is_device_memory(c->d_sc) || !is_device_memory(c->d_bins))
        return BUB_EINVAL;
    size_t off_sc, off_P, off_P2, ctx_bytes;
    ctx_buffer_layout(c->ndim, c->N, &off_sc, &off_P, &off_P2, &ctx_bytes);
    const size_t bytes = 3 * sizeof(double) * M + ctx_bytes;   // state, work, the context's buffers
    if (b->budget && b->used_bytes + bytes > b->budget) return BUB_ENOMEM;
    for (size_t i = 0; i < b->slots.size(); ++i) {
        auto &m = b->slots[i];
        if (!m.used) {
            m = bub_batch::Member{};
            m.ctx = c;
            m.q = q;
            m.work = work;
            m.used = true;
            m.bytes = bytes;
            m.remaining = steps;
            m.open = steps == 0;
            b->used_bytes += bytes;
            b->h_flags[i] = 0;
            b->dirty = true;
            const int t = batch_class_tile(b, c);
            if (t >= 0 && pw_fast(c)) c->tile = t;
            *slot = (int)i;
            return BUB_OK;
        }
    }
    return BUB_EINVAL;
}

int bub_batch_remove(bub_batch *b, int slot)
{
    if (!b || slot < 0 || slot >= (int)b->slots.size() || !b->slots[slot].used) return BUB_EINVAL;
    if (b->slots[slot].exec) b->retired.push_back(b->slots[slot].exec);   // launches may still be in flight
    b->used_bytes -= b->slots[slot].bytes;
    b->slots[slot] = bub_batch::Member{};
    b->dirty = true;
    return BUB_OK;
}

int bub_batch_info(const bub_batch *b, int *ncases, int64_t *cells, int64_t *cell_bins)
{
    if (!b) return BUB_EINVAL;
    int n = 0;
    long long cl = 0, cb = 0;
    for (auto &m : b->slots) {
        if (!m.used) continue;
        ++n;
        cl += m.ctx->N;
        cb += m.ctx->N * (long long)m.ctx->nb;
    }
    if (ncases) *ncases = n;
    if (cells) *cells = cl;
    if (cell_bins) *cell_bins = cb;
    return BUB_OK;
}

}  // extern "C"

namespace {

// nsteps steps of the members that `pick` selects, each member's own step kernels (or its captured
// step graph) on one of the batch's lanes, forked from and joined back into the caller's stream.
template <typename Pick>
int lanes_steps(bub_batch *b, int nsteps, hipStream_t s, Pick pick)
{
    // members, largest first, dealt to the least-loaded stream (work ~ cells x variables)
    std::vector<int> order;
    for (size_t i = 0; i < b->slots.size(); ++i)
        if (pick(b->slots[i])) order.push_back((int)i);
    if (order.empty() || nsteps == 0) return BUB_OK;
    auto work_of = [&](int i) { return (double)b->slots[i].ctx->N * (double)b->slots[i].ctx->nvar; };
    std::sort(order.begin(), order.end(), [&](int x, int y) { return work_of(x) > work_of(y); });
    double load[bub_batch::NSTREAM] = {};
    std::vector<int> lane(b->slots.size(), 0);
    for (int i : order) {
        int k = 0;
        for (int j = 1; j < b->lanes; ++j)
            if (load[j] < load[k]) k = j;
        lane[i] = k;
        load[k] += work_of(i);
    }
    const int used = (int)std::min<size_t>(order.size(), (size_t)b->lanes);
    if (b->retired.size() >= 64) {   // rare: wait for the lanes, then free removed members' graphs
        int rc = batch_free_retired(b);
        if (rc) return rc;
    }
    if (b->graphs)
        for (int i : order) {
            auto &m = b->slots[i];
            if (m.ctx->prof_on) continue;   // timed members launch directly
            if (!m.exec || m.cap_tile != m.ctx->tile || m.cap_groups != m.ctx->bin_groups) {
                int rc = batch_capture(b, m);
                if (rc) return rc;
            }
        }
    // fork: every lane starts after the work already queued on the caller's stream
    HIP_OK(hipEventRecord(b->fork, s));
    for (int k = 0; k < used; ++k) HIP_OK(hipStreamWaitEvent(b->st[k], b->fork, 0));
    // steps outer, members inner, so every lane's queue is fed from the start
    for (int step = 0; step < nsteps; ++step)
        for (int i : order) {
            auto &m = b->slots[i];
            if (b->graphs && m.exec && !m.ctx->prof_on) {
                HIP_OK(hipGraphLaunch(m.exec, b->st[lane[i]]));
            } else {
                int rc = bub_rk3_step(m.ctx, m.q, m.work, 0.0, nullptr, b->st[lane[i]]);
                if (rc) return rc;
            }
        }
    // join: the caller's stream continues after every lane
    for (int k = 0; k < used; ++k) {
        HIP_OK(hipEventRecord(b->join[k], b->st[k]));
        HIP_OK(hipStreamWaitEvent(s, b->join[k], 0));
    }
    return BUB_OK;
}

}  // namespace

extern "C" {

int bub_batch_step(bub_batch *b, int nsteps, void *stream)
{
    if (!b || nsteps < 0) return BUB_EINVAL;
    return lanes_steps(b, nsteps, (hipStream_t)stream, [](const bub_batch::Member &m) { return m.used; });
}

int bub_batch_graphs(bub_batch *b, int enable)
{
    if (!b) return BUB_EINVAL;
    b->graphs = enable != 0;
    return BUB_OK;
}

int bub_batch_lanes(bub_batch *b, int lanes)
{
    if (!b || lanes < 1 || lanes > bub_batch::NSTREAM) return BUB_EINVAL;
    b->lanes = lanes;
    return BUB_OK;
}

int bub_batch_tune_cache(bub_batch *b, const char *cache_path)
{
    if (!b) return BUB_EINVAL;
    b->tune_cache = cache_path ? cache_path : "";
    return BUB_OK;
}

int bub_batch_autotune(bub_batch *b, int reps, int *classes, void *stream)
{
    if (!b || reps < 1) return BUB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int tuned = 0;
    for (size_t i = 0; i < b->slots.size(); ++i) {
        auto &m = b->slots[i];
        if (!m.used || !pw_fast(m.ctx)) continue;   // the general power has one stage shape
        int t = batch_class_tile(b, m.ctx);
        if (t < 0) {
            // the cached shape of this class, or time the stage kernel's tile shapes on this member
            // (right-hand side into its work buffer)
            int rc = b->tune_cache.empty()
                         ? bub_autotune(m.ctx, m.q, m.work, reps, nullptr, &t, s)
                         : bub_autotune_cached(m.ctx, b->tune_cache.c_str(), m.q, m.work, reps, &t, nullptr, s);
            if (rc) return rc;
            b->tuned_key.emplace_back(m.ctx->ndim, m.ctx->nb);
            b->tuned_tile.push_back(t);
            ++tuned;
        }
        m.ctx->tile = t;
    }
    b->dirty = true;   // stage decompositions of the grouped launches follow the tiles
    if (classes) *classes = (int)b->tuned_key.size();
    (void)tuned;
    return BUB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Right-hand side for callers that cannot allocate: the context lives on the host stack and its
// device buffers (bin table, scalars, primitive scratch) in one file-scope device array
// ---------------------------------------------------------------------------

// Held by every GPU the library runs on until the process ends.  In host code `scratch` names a
// host-side stand-in: only the address from hipGetSymbolAddress is passed to kernels.
static __device__ __align__(256) unsigned char scratch[BUB_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per device (with it current).
int scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return BUB_EHIP;
    if (dev >= NOALLOC_MAX_DEVICES) return BUB_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BUB_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BUB_OK;
}

}  // namespace

extern "C" {

int bub_rhs_stage_noalloc(const bub_grid *grid, const bub_liquid *liq, const bub_gas *gas, const bub_bins *bins,
                          const bub_opts *opts, const double *q, double *rhs, int64_t *err, void *stream)
{
    if (!q || !rhs || q == rhs) return BUB_EINVAL;
    bub_ctx c;   // host side on the stack
    int rc = ctx_fill(grid, liq, gas, bins, opts, &c);
    if (rc) return rc;
    // bin table | scalars | one primitive scratch (a right-hand side needs no second one)
    size_t off_sc, off_P, off_P2, total;
    ctx_buffer_layout(c.ndim, c.N, &off_sc, &off_P, &off_P2, &total);
    const size_t need = off_P + sizeof(double) * (size_t)c.nprim * (size_t)c.N;
    if (need > BUB_NOALLOC_SCRATCH_BYTES) return BUB_ENOMEM;
    void *base_v = nullptr;
    if ((rc = scratch_address(&base_v))) return rc;
    char *base = (char *)base_v;
    c.owns = false;
    c.d_bins = (double *)base;
    c.d_sc = (Scalars *)(base + off_sc);
    c.d_P = (double *)(base + off_P);
    c.d_P2 = nullptr;
    ctx_finish(&c);
    hipStream_t s = (hipStream_t)stream;
    BinTable t{};
    bin_table(&c, t.v);
    // the previous call's contents are overwritten: bin table, cleared error word and maxima
    hipLaunchKernelGGL(k_ctx_init, dim3(1), dim3(64), 0, s, c.d_bins, t, 3 * c.nb, c.d_sc);
    HIP_OK(hipGetLastError());
    if ((rc = rhs_stage_impl(&c, q, rhs, s))) return rc;
    if (err) {
        hipLaunchKernelGGL(k_err_copy, dim3(1), dim3(64), 0, s, c.d_sc, err);
        HIP_OK(hipGetLastError());
    }
    return BUB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches, grouped form: one launch per phase and kernel class over a device member table
// ---------------------------------------------------------------------------
namespace {

constexpr int PRIM_CELLS_1 = 256, PRIM_CELLS_S = 64;   // cells per primitive/bubble block (as launch_prim)

int cells_for(int S) { return S == 1 ? PRIM_CELLS_1 : PRIM_CELLS_S; }

// The member's view for the grouped kernels; the stage decomposition is the one its own launch uses.
int member_desc(const bub_batch::Member &m, BatchMember *d)
{
    const bub_ctx *c = m.ctx;
    if (!pw_fast(c)) return BUB_EUNSUPPORTED;   // the grouped kernels carry the fifth-root power only
    *d = BatchMember{};
    const size_t M = (size_t)c->nvar * (size_t)c->N;
    d->q = m.q;
    d->w1 = m.work;
    d->w2 = m.work + M;
    d->P = c->d_P;
    d->sc = c->d_sc;
    d->g = c->g;
    d->ph = c->ph;
    d->bt = c->bt;
    d->cfl = c->opts.cfl;
    d->rtol = c->opts.sub_rtol > 0.0 ? c->opts.sub_rtol : 1e-4;
    d->max_substeps = c->opts.max_substeps > 0 ? c->opts.max_substeps : 10000;
    d->sources = c->opts.bubble_mode == BUB_BUBBLES_UNSPLIT;
    int tx, ty, tz, blk;
    if (bub_tile_info(c, c->tile, &tx, &ty, &tz, &blk)) return BUB_EINVAL;
    d->ntile[0] = (c->g.n[0] + tx - 1) / tx;
    d->ntile[1] = (c->g.n[1] + ty - 1) / ty;
    d->ntile[2] = (c->g.n[2] + tz - 1) / tz;
    d->ntiles = d->ntile[0] * d->ntile[1] * d->ntile[2];
    d->bpg = bin_grouping(c, d->ntiles, &d->ngroups);
    d->nitems = d->ntiles * d->ngroups;
    return BUB_OK;
}

bool member_active(const bub_batch::Member &m) { return m.used && (m.open || m.remaining > 0); }

// Rewrite the member table and the launch lists for the members still stepping: both are filled in
// the next staging buffer of the ring (once the upload that last read it has completed) and uploaded
// on the batch's stream, ahead of the chunk that reads them.
int batch_rebuild(bub_batch *b, hipStream_t s)
{
    const int r = b->stage_next;
    if (b->stage_used[r]) HIP_OK(hipEventSynchronize(b->stage_ev[r]));
    BatchMember *tab = reinterpret_cast<BatchMember *>(b->h_stage[r]);
    LaunchList *lists = reinterpret_cast<LaunchList *>(b->h_stage[r] + sizeof(BatchMember) * b->slots.size());
    std::vector<PlanMember> pm;
    for (size_t i = 0; i < b->slots.size(); ++i) {
        const auto &m = b->slots[i];
        if (!member_active(m)) continue;
        int rc = member_desc(m, &tab[i]);
        if (rc) return rc;
        const bub_ctx *c = m.ctx;
        const int S = slots_for(c->N);
        pm.push_back({(int)i, c->ndim, S, c->tile, c->opts.bubble_mode == BUB_BUBBLES_SPLIT,
                      (c->N + cells_for(S) - 1) / cells_for(S), (long long)tab[i].nitems});
    }
    BatchPlan plan;
    if (plan_batch(pm, bub_batch::NLISTS, &plan)) return BUB_EUNSUPPORTED;
    for (size_t k = 0; k < plan.lists.size(); ++k) lists[k] = plan.lists[k];
    HIP_OK(hipMemcpyAsync(b->d_tab, tab, sizeof(BatchMember) * b->slots.size(), hipMemcpyHostToDevice, s));
    if (!plan.lists.empty())
        HIP_OK(hipMemcpyAsync(b->d_lists, lists, sizeof(LaunchList) * plan.lists.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipEventRecord(b->stage_ev[r], s));
    b->stage_used[r] = true;
    b->stage_next = (r + 1) % bub_batch::NSTAGE;
    auto conv = [](const std::vector<PlanLaunch> &v) {
        std::vector<bub_batch::Launch> o;
        for (const auto &l : v) o.push_back({l.d, l.key, l.list, l.blocks});
        return o;
    };
    b->prim_all = conv(plan.prim_all);
    b->prim_split = conv(plan.prim_split);
    b->stage_l = conv(plan.stage);
    b->dt_list = plan.dt_list;
    b->dt_count = plan.dt_count;
    b->dirty = false;
    ++b->version;
    return BUB_OK;
}

template <int D, int MODE>
void launch_prim_group(const bub_batch *b, const bub_batch::Launch &l, int which, hipStream_t s)
{
    const dim3 grid((unsigned)l.blocks);
    const LaunchList *L = b->d_lists + l.list;
    switch (l.key) {
    case 1: hipLaunchKernelGGL((k_prim_group<D, MODE, 1, PRIM_CELLS_1>), grid, dim3(PRIM_CELLS_1), 0, s, b->d_tab, L, which); break;
    case 2: hipLaunchKernelGGL((k_prim_group<D, MODE, 2, PRIM_CELLS_S>), grid, dim3(2 * PRIM_CELLS_S), 0, s, b->d_tab, L, which); break;
    case 4: hipLaunchKernelGGL((k_prim_group<D, MODE, 4, PRIM_CELLS_S>), grid, dim3(4 * PRIM_CELLS_S), 0, s, b->d_tab, L, which); break;
    default: hipLaunchKernelGGL((k_prim_group<D, MODE, 8, PRIM_CELLS_S>), grid, dim3(8 * PRIM_CELLS_S), 0, s, b->d_tab, L, which); break;
    }
}

void prim_groups(const bub_batch *b, const std::vector<bub_batch::Launch> &v, int which, bool cfl, hipStream_t s)
{
    for (const auto &l : v) {
        if (l.d == 1) cfl ? launch_prim_group<1, PRIM_CFL>(b, l, which, s) : launch_prim_group<1, PRIM_ONLY>(b, l, which, s);
        else if (l.d == 2) cfl ? launch_prim_group<2, PRIM_CFL>(b, l, which, s) : launch_prim_group<2, PRIM_ONLY>(b, l, which, s);
        else cfl ? launch_prim_group<3, PRIM_CFL>(b, l, which, s) : launch_prim_group<3, PRIM_ONLY>(b, l, which, s);
    }
}

template <int D>
void launch_bubble_group(const bub_batch *b, const bub_batch::Launch &l, hipStream_t s)
{
    const dim3 grid((unsigned)l.blocks);
    const LaunchList *L = b->d_lists + l.list;
    switch (l.key) {
    case 1: hipLaunchKernelGGL((k_bubble_group<D, 1, PRIM_CELLS_1>), grid, dim3(PRIM_CELLS_1), 0, s, b->d_tab, L); break;
    case 2: hipLaunchKernelGGL((k_bubble_group<D, 2, PRIM_CELLS_S>), grid, dim3(2 * PRIM_CELLS_S), 0, s, b->d_tab, L); break;
    case 4: hipLaunchKernelGGL((k_bubble_group<D, 4, PRIM_CELLS_S>), grid, dim3(4 * PRIM_CELLS_S), 0, s, b->d_tab, L); break;
    default: hipLaunchKernelGGL((k_bubble_group<D, 8, PRIM_CELLS_S>), grid, dim3(8 * PRIM_CELLS_S), 0, s, b->d_tab, L); break;
    }
}

void bubble_groups(const bub_batch *b, hipStream_t s)
{
    for (const auto &l : b->prim_split) {
        if (l.d == 1) launch_bubble_group<1>(b, l, s);
        else if (l.d == 2) launch_bubble_group<2>(b, l, s);
        else launch_bubble_group<3>(b, l, s);
    }
}

template <int D, int V, typename TF>
void launch_stage_group_t(const bub_batch *b, const bub_batch::Launch &l, int stage, hipStream_t s)
{
    using TC = Tile<D, V>;
    const int per_xcd = (int)((l.blocks + 7) / 8);
    hipLaunchKernelGGL((k_stage_group<D, TC::TX, TC::TY, TC::TZ, TC::BLOCK, TF>), dim3(8 * per_xcd), dim3(TC::BLOCK),
                       0, s, b->d_tab, b->d_lists + l.list, stage, per_xcd);
}

template <int D, int V>
void launch_stage_group_v(const bub_batch *b, const bub_batch::Launch &l, int stage, hipStream_t s)
{
    if (b->precision == BUB_PREC_MIXED) launch_stage_group_t<D, V, float>(b, l, stage, s);
    else launch_stage_group_t<D, V, double>(b, l, stage, s);
}

void stage_groups(const bub_batch *b, int stage, hipStream_t s)
{
    for (const auto &l : b->stage_l) {
        const int v = l.key;
        switch (l.d) {
        case 1:
            if (v == 1) launch_stage_group_v<1, 1>(b, l, stage, s);
            else if (v == 2) launch_stage_group_v<1, 2>(b, l, stage, s);
            else launch_stage_group_v<1, 0>(b, l, stage, s);
            break;
        case 2:
            if (v == 1) launch_stage_group_v<2, 1>(b, l, stage, s);
            else if (v == 2) launch_stage_group_v<2, 2>(b, l, stage, s);
            else if (v == 3) launch_stage_group_v<2, 3>(b, l, stage, s);
            else if (v == 4) launch_stage_group_v<2, 4>(b, l, stage, s);
            else if (v == 5) launch_stage_group_v<2, 5>(b, l, stage, s);
            else launch_stage_group_v<2, 0>(b, l, stage, s);
            break;
        default:
            if (v == 1) launch_stage_group_v<3, 1>(b, l, stage, s);
            else if (v == 2) launch_stage_group_v<3, 2>(b, l, stage, s);
            else if (v == 3) launch_stage_group_v<3, 3>(b, l, stage, s);
            else if (v == 4) launch_stage_group_v<3, 4>(b, l, stage, s);
            else launch_stage_group_v<3, 0>(b, l, stage, s);
            break;
        }
    }
}

// nsteps CFL-limited SSP-RK3 steps of every listed member: the phases of bub_rk3_step, each one
// launch per kernel class for all members (split members add their bubble half-steps).
int batch_chunk(const bub_batch *b, int nsteps, hipStream_t s)
{
    const bool any_split = !b->prim_split.empty();
    for (int k = 0; k < nsteps; ++k) {
        prim_groups(b, b->prim_all, 0, true, s);                      // primitives and wave speeds of u^n
        hipLaunchKernelGGL(k_dt_group, dim3((unsigned)b->dt_count), dim3(WMAX_SLOTS), 0, s, b->d_tab,
                           b->d_lists + b->dt_list);
        if (any_split) {
            bubble_groups(b, s);                                         // S_b(dt/2)
            prim_groups(b, b->prim_split, 0, false, s);
        }
        stage_groups(b, 1, s);
        prim_groups(b, b->prim_all, 1, false, s);
        stage_groups(b, 2, s);
        prim_groups(b, b->prim_all, 2, false, s);
        stage_groups(b, 3, s);
        if (any_split) bubble_groups(b, s);                              // S_b(dt/2)
    }
    return hipGetLastError() == hipSuccess ? BUB_OK : BUB_EHIP;
}

// Capture a chunk of nsteps into one graph (kernels only) unless the cached one matches.
int batch_chunk_graph(bub_batch *b, int nsteps)
{
    if (b->run_exec && b->run_steps == nsteps && b->run_version == b->version) return BUB_OK;
    hipGraph_t g = nullptr;
    HIP_OK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const int rc = batch_chunk(b, nsteps, b->cap);
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : BUB_EHIP;
    }
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return BUB_EHIP;
    if (b->run_exec) {   // an earlier launch of it may still run: free it once its last launch is done
        b->run_retired.emplace_back(b->run_exec, b->run_ev);
        b->run_ev = nullptr;
    }
    if (!b->run_ev && hipEventCreateWithFlags(&b->run_ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGraphExecDestroy(x);
        b->run_exec = nullptr;
        return BUB_EHIP;
    }
    b->run_exec = x;
    b->run_steps = nsteps;
    b->run_version = b->version;
    return BUB_OK;
}

}  // namespace

extern "C" {

int bub_batch_run(bub_batch *b, int max_steps, int *steps_taken, void *stream)
{
    if (!b || max_steps < 0) return BUB_EINVAL;
    if (steps_taken) *steps_taken = 0;
    hipStream_t s = (hipStream_t)stream;
    // the chunk: at most max_steps, never past the member with the fewest steps left
    int n = max_steps;
    bool any = false;
    for (const auto &m : b->slots) {
        if (!member_active(m)) continue;
        any = true;
        if (!m.open && m.remaining < n) n = m.remaining;
    }
    if (!any || n == 0) return BUB_OK;
    int rc;
    if (kGroupedLaunches) {
        if (b->dirty && (rc = batch_rebuild(b, s))) return rc;
        for (size_t k = 0; k < b->run_retired.size();) {
            if (hipEventQuery(b->run_retired[k].second) == hipSuccess) {
                (void)hipGraphExecDestroy(b->run_retired[k].first);
                (void)hipEventDestroy(b->run_retired[k].second);
                b->run_retired[k] = b->run_retired.back();
                b->run_retired.pop_back();
            } else {
                ++k;
            }
        }
        if (b->graphs) {
            if ((rc = batch_chunk_graph(b, n))) return rc;
            HIP_OK(hipGraphLaunch(b->run_exec, s));
            HIP_OK(hipEventRecord(b->run_ev, s));
        } else if ((rc = batch_chunk(b, n, s))) {
            return rc;
        }
    } else if ((rc = lanes_steps(b, n, s, member_active))) {
        return rc;
    }
    // members whose last step is now queued: a flag in host memory marks their completion
    ++b->epoch;
    for (size_t i = 0; i < b->slots.size(); ++i) {
        auto &m = b->slots[i];
        if (!member_active(m) || m.open) continue;
        m.remaining -= n;
        if (m.remaining == 0) {
            m.done_epoch = b->epoch;
            hipLaunchKernelGGL(k_flag_set, dim3(1), dim3(64), 0, s, b->d_flags, (int)i, b->epoch);
            b->dirty = true;   // finished members leave the lists
        }
    }
    HIP_OK(hipGetLastError());
    if (steps_taken) *steps_taken = n;
    return BUB_OK;
}

int bub_batch_poll(bub_batch *b, int *done_slots, int *ndone)
{
    if (!b || !ndone || !done_slots) return BUB_EINVAL;
    int k = 0;
    for (size_t i = 0; i < b->slots.size(); ++i) {
        auto &m = b->slots[i];
        if (!m.used || m.reported || m.done_epoch == 0) continue;
        if (__atomic_load_n(&b->h_flags[i], __ATOMIC_ACQUIRE) == m.done_epoch) {
            m.reported = true;
            done_slots[k++] = (int)i;
        }
    }
    *ndone = k;
    return BUB_OK;
}

int bub_batch_remaining(const bub_batch *b, int slot, int *steps)
{
    if (!b || !steps || slot < 0 || slot >= (int)b->slots.size() || !b->slots[slot].used) return BUB_EINVAL;
    *steps = b->slots[slot].open ? -1 : b->slots[slot].remaining;
    return BUB_OK;
}

}  // extern "C"
