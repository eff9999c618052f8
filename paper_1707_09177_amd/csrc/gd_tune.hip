// gd_tune.hip -- tile-shape selection for the stencil sweeps.
//
// A tile is one wavefront's unit of work: 64 lanes x vw columns, R rows (3D)
// and L planes along the march axis.  Wider lanes (16-byte loads) need nx to be
// a multiple of the vector width and 16-byte aligned fields.  The halo cost of
// a tile is 2/L extra planes along the march axis and, in 3D, 2/R extra rows
// (those mostly hit L2 because neighbouring tiles run on the same XCD).  L is
// picked so that the batch yields enough tiles to keep every wave of the chip
// busy: MI355X runs up to 256 CUs x 16 waves of this kernel.
#include <algorithm>

#include "gd_internal.h"

namespace gd {

namespace {
constexpr int64_t kWaveSlots = 256 * 16;  // resident waves assumed before the kernel is known
}

// Lane width and rows per tile.
TileShape choose_tiles(int ndim, int64_t nx, int64_t ny, int64_t nz, int64_t batch, int tsize, bool aligned,
                       int /*solver*/, bool mixed) {
    TileShape t;
    const int vmax = 16 / tsize;
    t.vw = (aligned && nx % vmax == 0 && nx >= vmax) ? vmax : 1;
    t.blocks_per_cu = 0;
    if (ndim == 2) {
        t.R = 1;
    } else if (t.vw > 1) {
        t.R = ny >= 2 ? 2 : 1;
    } else {
        t.R = (!mixed && ny >= 4) ? 4 : 1;
    }
    t.L = balanced_L(ndim == 2 ? ny : nz, batch * tiles_per_plane(ndim, nx, ny, t.vw, t.R), kWaveSlots);
    return t;
}

int64_t tiles_per_plane(int ndim, int64_t nx, int64_t ny, int vw, int R) {
    const int64_t tc = ndim == 3 ? tile_cols(vw, R) : 64 * vw;  // x columns per tile
    const int64_t nxs = (nx + tc - 1) / tc;
    return ndim == 2 ? nxs : nxs * ((ny + R - 1) / R);
}

// Planes per tile for `cols` independent tile columns of `nmarch` planes run
// by `waves` resident waves (tile t goes to wave t mod waves).  Minimises the
// planes the busiest wave marches, halo planes included, preferring longer
// tiles on ties (fewer halo re-reads).
int64_t balanced_L(int64_t nmarch, int64_t cols, int64_t waves) {
    waves = std::max<int64_t>(1, waves);
    cols = std::max<int64_t>(1, cols);
    int64_t bestL = std::max<int64_t>(1, std::min<int64_t>(nmarch, kMaxL));
    int64_t bestCost = INT64_MAX;
    const int64_t nseg_max = std::max<int64_t>(1, (nmarch + kMinL - 1) / kMinL);
    for (int64_t nseg = 1; nseg <= nseg_max; ++nseg) {
        const int64_t L = (nmarch + nseg - 1) / nseg;
        if (L > kMaxL || (L < kMinL && nseg > 1)) continue;
        const int64_t segs = (nmarch + L - 1) / L;
        const int64_t tiles = cols * segs;
        const int64_t per_wave = (tiles + waves - 1) / waves;
        const int64_t cost = per_wave * (L + 2);
        if (cost < bestCost || (cost == bestCost && L > bestL)) {
            bestCost = cost;
            bestL = L;
        }
    }
    return std::max<int64_t>(kMinL, bestL);
}

}  // namespace gd
