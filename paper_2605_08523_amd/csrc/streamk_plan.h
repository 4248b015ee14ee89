// Work split of the stream-K schedules of the 16-bit layer kernel, shared by the kernel (device)
// and by the host (the launcher, and fe_streamk_segments, which lets a CPU test walk the same
// code that the kernel runs).
//
// The upper tiles [dp_tiles, ntiles) of one layer, times their nk K-blocks each, form a list of
// (tile, K-block) iterations. The grid is split into `groups` groups (8: one per XCD, since the
// hardware hands consecutive workgroups to consecutive XCDs, so the workgroups w with one value of
// w % 8 share an XCD); group g owns a contiguous run of those tiles and
// deals its iterations to its GX = grid / groups workgroups in contiguous, near-equal ranges.
// A workgroup whose range stops inside a tile publishes that partial tile; the workgroup that
// reaches the tile's last K-block adds the earlier contributors' partials in a fixed order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fe {

struct SkGeometry {
    int T;          // tiles per side of the padded matrix
    int ntiles;     // upper tiles, T (T + 1) / 2
    int nk;         // K-blocks per tile
    int dp_tiles;   // leading tiles computed whole by a data-parallel launch before this one
    int groups;     // workgroup groups (1 or 8)
    int grid;       // stream-K workgroups
};

// Plan of one stream-K launch: np padded size, bm x bm tiles, bk-deep K-blocks, at most
// `grid` workgroups. With two or more full rounds of tiles and register-held accumulators
// (reg_epi), all but the last round run whole in a data-parallel launch first. Eight groups when
// every group gets at least one tile and at least one iteration per workgroup, else one group
// with at most one workgroup per iteration: every range is then non-empty.
__host__ __device__ inline SkGeometry sk_plan(int64_t np, int bm, int bk, int grid, bool reg_epi) {
    SkGeometry G;
    G.T = (int)(np / bm);
    G.ntiles = G.T * (G.T + 1) / 2;
    G.nk = (int)(np / bk);
    const int64_t rounds = G.ntiles / grid;
    G.dp_tiles = (reg_epi && rounds >= 2) ? (int)((rounds - 1) * grid) : 0;
    const int64_t nsk = G.ntiles - G.dp_tiles;
    G.grid = grid;
    if (nsk >= 8 && grid % 8 == 0 && (nsk / 8) * G.nk >= grid / 8) {
        G.groups = 8;
    } else {
        G.groups = 1;
        if ((int64_t)G.grid > nsk * G.nk) G.grid = (int)(nsk * G.nk);
    }
    return G;
}

// First iteration of workgroup index jj of a group whose iterations are [base, base + total).
__host__ __device__ inline int64_t sk_range_start(int64_t base, int64_t total, int jj, int GX) {
    return base + total * jj / GX;
}

// Segments of workgroup w, in the order the kernel runs them; f(pass, t, kb0, kb1, jlo) is called
// for each: tile t, K-blocks [kb0, kb1). Passes:
//  0: if the range stops inside its last tile, that tail, published first so that the workgroup
//     finishing that tile never waits behind this one (no chains of waits across the grid);
//  1: the segments that start on a tile boundary and finish their tile (no waiting);
//  2: if the range starts inside a tile, the rest of that tile, which waits for the earlier
//     workgroups' partials: last, so that they have had the longest time to publish.
// For passes 1 and 2 with kb0 > 0, the group's workgroups with indices jlo .. j - 1 (ids
// g + groups jj) hold blocks [0, kb0) of the tile as published partials; otherwise jlo = j.
template <class F>
__host__ __device__ __attribute__((always_inline)) inline void sk_walk(const SkGeometry& G, int w,
                                                                       F&& f) {
    const int nk = G.nk;
    const int t0 = G.dp_tiles, nsk = G.ntiles - G.dp_tiles;
    const int NG = G.groups, g = w % NG, j = w / NG, GX = G.grid / NG;
    const int tg0 = t0 + (int)((int64_t)nsk * g / NG), tg1 = t0 + (int)((int64_t)nsk * (g + 1) / NG);
    const int64_t base = (int64_t)tg0 * nk, total = (int64_t)(tg1 - tg0) * nk;
    const int64_t a_w = sk_range_start(base, total, j, GX), b_w = sk_range_start(base, total, j + 1, GX);
    const int t_last = (int)((b_w - 1) / nk);
    const int64_t tail_start = (int64_t)t_last * nk > a_w ? (int64_t)t_last * nk : a_w;
    const bool publishes = b_w < (int64_t)(t_last + 1) * nk;
    const int64_t own_end = publishes ? tail_start : b_w;
    const int64_t a_up = (a_w + nk - 1) / nk * nk;
    const int64_t first_boundary = a_up < own_end ? a_up : own_end;
    for (int pass = publishes ? 0 : 1; pass < 3; ++pass) {
        int64_t it = pass == 0 ? tail_start : pass == 1 ? first_boundary : a_w;
        const int64_t stop = pass == 0 ? b_w : pass == 1 ? own_end : first_boundary;
        while (it < stop) {
            const int t = (int)(it / nk);
            const int kb0 = (int)(it - (int64_t)t * nk);
            const int64_t rest = stop - it;
            const int kb1 = (int)((int64_t)kb0 + rest < nk ? kb0 + rest : nk);
            int jlo = j;
            if (pass != 0 && kb0 > 0)
                while (jlo > 0 && sk_range_start(base, total, jlo, GX) > (int64_t)t * nk) --jlo;
            f(pass, t, kb0, kb1, jlo);
            it += kb1 - kb0;
        }
    }
}

}  // namespace fe
