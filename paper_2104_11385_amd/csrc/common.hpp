// Internal declarations shared by the library's HIP and host sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "picbal.h"

namespace pb {

constexpr int kMaxSpecies = 4;
constexpr int kSubQueues = 8;   // one persistent work sub-queue per XCD

// Particle cell index packed in 32 bits: x in bits 0..10, y in 11..21,
// z in 22..31 (domain up to 2048 x 2048 x 1024 cells).
__host__ __device__ inline uint32_t pack_cell(int x, int y, int z) {
    return (uint32_t)x | ((uint32_t)y << 11) | ((uint32_t)z << 22);
}
__host__ __device__ inline void unpack_cell(uint32_t c, int &x, int &y, int &z) {
    x = (int)(c & 2047u);
    y = (int)((c >> 11) & 2047u);
    z = (int)(c >> 22);
}

// Structure-of-arrays particle storage.  A particle's position is its cell
// (packed) plus an offset f in [0, 1) per dimension, so that a 32-bit float
// keeps ~6e-8 cell of resolution everywhere in the domain and the shape
// factors of the current deposit are formed without cancellation.
template <typename real>
struct Particles {
    uint32_t *cell;
    real *f[3];
    real *u[3];
    real *w;
    int64_t *id;
    uint8_t *sp;
};

// Tile origin (global cell coordinates of its lowest corner), owning box,
// and that box's lowest and highest cell, packed like a particle's cell.
struct TileDesc {
    int x0, y0, z0, box;
    uint32_t box_lo, box_hi;
};

// Geometry needed to map a cell to (box, tile, cell-in-tile).
struct Geom {
    int n[3];
    int T[3];
    int Tvol;
    int g[3];            // coarse granularity (gcd of box corners per dim)
    int cg[3];           // coarse grid dims
    const int *coarse_box;   // box of each coarse cell
    const int *box_lo;       // [nb][3]
    const int *box_nt;       // tiles per dim [nb][3]
    const int *box_tile_off; // [nb+1]
    int nsp;
    int order;
};

enum { MODE_PER_BOX = 0, MODE_BATCHED = 1, MODE_PERSISTENT = 2 };

// Box bounds and the cell -> box lookup, in device memory (read by the
// gather-push-deposit kernel only for particles outside their tile's box).
struct BoxMap {
    const int *boxes6;       // [nb][6] lo, hi of each box
    const int *coarse_box;   // box of each coarse cell (cell / g)
    int g[3], cg[3];         // coarse cell edge and coarse grid size
};

// Arguments of the gather-push-deposit kernel.
template <typename real>
struct GpdArgs {
    Particles<real> P;
    const int *segstart;       // [ntiles*nsp + 1] particle ranges per (tile, species)
    const TileDesc *tiles;
    const real *EB[6];         // Ex Ey Ez Bx By Bz
    real *J[3];
    int n[3];
    int nsp;
    real dt;
    real bext[3];              // uniform external B, added at the gather
    real h[kMaxSpecies];       // q dt / (2 m)
    real coefq[kMaxSpecies];   // -q / dt
    unsigned long long *cycles;    // [nb]
    unsigned long long *rtc;       // [nb]
    const BoxMap *bmap;            // box bounds and the cell -> box map
    unsigned int *slow;            // particles that took the global path
    int *slowlist;                 // [capacity] particles left to the global-path kernel
    unsigned int *slown;           // [2] entries in slowlist, and blocks of the global kernel done
    int *jdirty;                   // [n[2]] set to 1 for every z-plane of J written
    int mode;
    int timer;                 // nonzero: per-box clock counters are updated
    int tile_base;             // PER_BOX: first tile of the box
    int species_only;          // PER_BOX: species of this launch
    const int4 *queue;         // PERSISTENT: (tile, begin, end, -)
    const int *queue_bounds;   // [kSubQueues + 1] sub-queue ranges
    int *queue_head;           // [kSubQueues] next item of each sub-queue
};

}  // namespace pb
