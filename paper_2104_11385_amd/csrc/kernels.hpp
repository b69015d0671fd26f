// Host-side launchers of the PIC kernels (implemented in pic_kernels.hip).
#pragma once

#include <algorithm>

#include "common.hpp"

namespace pb {

// Precision-erased particle arrays.
struct ParticlesRaw {
    uint32_t *cell = nullptr;
    void *f[3] = {nullptr, nullptr, nullptr};
    void *u[3] = {nullptr, nullptr, nullptr};
    void *w = nullptr;
    int64_t *id = nullptr;
    uint8_t *sp = nullptr;
};

// On-device loader of one species (recipe: Philox4x32-10 words -> cell
// offsets and Box-Muller normals; see the Python input generator).
struct LoadArgs {
    int mode;                 // 1: fixed ppc in a region, 2: per-box ppc
    int rlo[3], rext[3];
    int ppc;
    const int64_t *box_base;  // [nb+1] prefix of cells*ppc (mode 2)
    const int32_t *box_ppc;   // [nb]
    const int *boxes6;        // [nb][6]
    int nb;
    int64_t n;                // particles of this species
    int64_t out_base;         // first slot in the particle arrays
    int species;
    uint32_t k0, k1;          // Philox key
    double uth[3], udrift[3];
    double density;
};

struct SortScratch {
    int nseg;                 // ntiles * nsp
    uint32_t *cellcnt;        // [nseg * Tvol]
    uint32_t *cellstart;      // [nseg * Tvol]
    int *segtot;              // [nseg]
    int *segstart;            // [nseg + 1]
    uint32_t *key, *rank;     // [capacity]
    uint32_t *table;          // [capacity]
    int *bsum, *boff;         // [nseg / 1024 + 2] block sums for the segment scan
};

struct QueueScratch {
    int ncls;
    int *cls_cnt;             // [kSubQueues * ncls]
    int *cursor;              // [kSubQueues * ncls]
    int *queue_bounds;        // [kSubQueues + 1]
    int *queue_head;          // [kSubQueues]
    int4 *queue;              // [max items]
};

struct FeatScratch {
    uint32_t *cellcount;      // [n cells]
    unsigned long long *spcnt;    // [nb][2]
    unsigned long long *edge;     // [nb]
    double *usum;                 // [nb]
};

struct GpdLaunch {
    ParticlesRaw P;
    const int *segstart;
    const TileDesc *tiles;
    const void *EB[6];
    void *J[3];
    int n[3];
    int nsp;
    double dt;
    double bext[3];
    double h[kMaxSpecies];
    double coefq[kMaxSpecies];
    unsigned long long *cycles, *rtc;
    const BoxMap *bmap;        // device copy of the box bounds and map
    unsigned int *slow;
    int *slowlist;             // [capacity] list of the particles left to the global-path kernel
    unsigned int *slown;       // [2] its length and a completion counter (zero between steps)
    int *jdirty;               // [nz] z-planes of J the deposit touched
    int mode;
    int timer;
    int staged;                // zero: every particle through the global-path kernel
    int tile_base;
    int species_only;
    const int4 *queue;
    const int *queue_bounds;
    int *queue_head;
    int tile[3];
    int halo;
    int run_sum;               // kept-node currents summed over lane runs
    unsigned grid, block;
    int *regs_out;             // non-null: receives the kernel's VGPRs per lane (grid 0: query only)
};

hipError_t launch_load(int prec, const ParticlesRaw &P, const LoadArgs &a, hipStream_t st);
hipError_t launch_sort(int prec, const ParticlesRaw &S, const ParticlesRaw &D, int np, const Geom &G,
                       const SortScratch &W, bool node_major, hipStream_t st);
hipError_t launch_queue(const int *segstart, int ntiles, int nsp, int chunk, const QueueScratch &Q, hipStream_t st);
hipError_t launch_set_int(int *p, int v, hipStream_t st);
hipError_t launch_fill_f(int prec, void *a, double v, size_t n, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *a, size_t n, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *a, size_t n, hipStream_t st, uint32_t v = 0);
hipError_t launch_fill_f64(double *a, size_t n, hipStream_t st);
hipError_t launch_gpd(int prec, int order, const GpdLaunch &L, hipStream_t st);
// The global path: over the tile kernels' list (n < 0), or every particle
// [0, n) (staging off); grid blocks of 256 threads.
hipError_t launch_gpd_global(int prec, int order, const GpdLaunch &L, int n, unsigned grid, hipStream_t st);
bool gpd_supported(const int tile[3], int halo);
size_t gpd_lds_bytes(int prec, int order, const int tile[3], int halo, int block);
// Field buffers of one Yee update: inputs E, B, J; outputs Eo, Bo; Z is the
// J buffer cleared for the next deposit.
// Fields of one Yee update: inputs E, B, J; X holds B^{n+1/2} on entry to
// launch_yee (launch_yee_half computes it from E and B) and B^{n+3/2} on
// exit; outputs Eo, Bo; Z is the J buffer cleared for the next deposit.
// jdirty / zdirty: per z-plane occupancy flags of J and Z (0: the plane is
// zero); the second part of launch_yee resets zdirty.  lists: [4 nz + 4]
// plane lists and counts written by launch_yee_class.
struct YeeBuffers {
    const void *E[3], *B[3], *J[3];
    void *X[3];
    void *Eo[3], *Bo[3], *Z[3];
    const int *jdirty;
    int *zdirty;
    int *lists;
};
hipError_t launch_yee_half(int prec, const YeeBuffers &Y, const int n[3], double dt, hipStream_t st);
// Splits the z-planes into those no deposit of the coming step reaches (all
// planes go to the second part when split is false); with heads non-null it
// also zeroes the persistent queue's kSubQueues sub-queue heads.
hipError_t launch_yee_class(const YeeBuffers &Y, int nz, bool split, int *heads, hipStream_t st);
// E and B passes of one part: 0 the planes out of the deposit's reach (may
// run beside the particle kernel), 1 the rest (after it); grid blocks.
hipError_t launch_yee(int prec, const YeeBuffers &Y, const int n[3], double dt, int part, unsigned grid,
                      hipStream_t st);
hipError_t launch_find_ids(int prec, const ParticlesRaw &P, int np, int s, const int64_t *q, int n, uint32_t *cell,
                           void *f, void *u, int *found, hipStream_t st);
hipError_t launch_box_counts(int prec, const ParticlesRaw &P, int np, const Geom &G, unsigned long long *counts,
                             hipStream_t st);
hipError_t launch_features(int prec, const ParticlesRaw &P, int np, const Geom &G, int nb, const int *box_hi,
                           const FeatScratch &S, float *feat, hipStream_t st);

}  // namespace pb
