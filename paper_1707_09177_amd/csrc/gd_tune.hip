// gd_tune.cpp -- tile-shape selection for the stencil sweeps.
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
constexpr int64_t kWaveSlots = 256 * 16;  // resident waves we aim to fill
}

TileShape choose_tiles(int ndim, int64_t nx, int64_t ny, int64_t nz, int64_t batch, int tsize, bool aligned,
                       int /*solver*/, bool mixed) {
    TileShape t;
    const int vmax = 16 / tsize;
    t.vw = (aligned && nx % vmax == 0 && nx >= vmax) ? vmax : 1;
    t.blocks_per_cu = 0;
    int64_t nmarch;
    int64_t per_plane;
    const int64_t nxs = (nx + 64 * t.vw - 1) / (64 * t.vw);
    if (ndim == 2) {
        t.R = 1;
        nmarch = ny;
        per_plane = nxs;
    } else {
        if (t.vw > 1) t.R = ny >= 2 ? 2 : 1;
        else t.R = (!mixed && ny >= 4) ? 4 : 1;
        nmarch = nz;
        per_plane = nxs * ((ny + t.R - 1) / t.R);
    }
    // planes per tile: as long as possible while still giving >= 2 tiles per
    // resident wave; never below kMinL, never above 256
    const int64_t want_tiles = 2 * kWaveSlots;
    int64_t L = (batch * per_plane * nmarch) / std::max<int64_t>(1, want_tiles);
    L = std::max<int64_t>(kMinL, std::min<int64_t>(256, L));
    L = std::min<int64_t>(L, std::max<int64_t>(kMinL, nmarch));
    t.L = L;
    return t;
}

}  // namespace gd
