// Device helpers shared by the PIC kernels: periodic wraps, single-precision
// hardware reciprocals, atomics, block scans, wave-aggregated counters and
// the box / tile lookup of a cell.
#pragma once

#include "common.hpp"

#include <hip/hip_runtime.h>

namespace pb {

__device__ __forceinline__ int wrap_any(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// Wraps i into [0, n) when it lies in [-n, 2n) (one conditional step).
__device__ __forceinline__ int wrap_near(int i, int n) {
    i = i < 0 ? i + n : i;
    return i >= n ? i - n : i;
}

// Wraps a tile-relative coordinate r into [-h, n - h).
__device__ __forceinline__ int wrap_rel(int r, int h, int n) {
    int t = r + h;
    if (t < 0) t += n;
    else if (t >= n) t -= n;
    if (t < 0 || t >= n) t = wrap_any(t, n);
    return t - h;
}

// 1/sqrt(x) and 1/x: the hardware approximations (about 1 ulp) in single
// precision, correctly rounded operations in double precision.
__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_r(double x) { return 1.0 / x; }

template <typename real>
__device__ __forceinline__ void atomic_add_global(real *p, real v) {
    unsafeAtomicAdd(p, v);
}

template <typename real>
__device__ __forceinline__ void atomic_add_lds(real *p, real v) {
    unsafeAtomicAdd(p, v);
}

// Exclusive block scan of one int per thread (blockDim a multiple of 64,
// at most 1024).  sh needs 17 ints.  Returns the exclusive prefix; total is
// the block sum.
__device__ inline int block_excl_scan(int v, int *sh, int &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < nw; ++i) {
            int t = sh[i];
            sh[i] = acc;
            acc += t;
        }
        sh[16] = acc;
    }
    __syncthreads();
    int r = x - v + sh[wid];
    total = sh[16];
    __syncthreads();
    return r;
}

// Adds 1 to arr[key] for every active lane, with one atomic per distinct key
// in the wave.
__device__ inline void wave_count_add(unsigned long long *arr, int key) {
    unsigned long long active = __ballot(1);
    while (active) {
        int leader = __ffsll((long long)active) - 1;
        int lkey = __shfl(key, leader);
        unsigned long long same = __ballot(key == lkey) & active;
        if (key == lkey && (int)__lane_id() == leader)
            atomicAdd(&arr[key], (unsigned long long)__popcll(same));
        active &= ~same;
    }
}

__device__ inline void wave_sum_add(double *arr, int key, double v) {
    unsigned long long active = __ballot(1);
    while (active) {
        int leader = __ffsll((long long)active) - 1;
        int lkey = __shfl(key, leader);
        bool mine = key == lkey;
        unsigned long long same = __ballot(mine) & active;
        double s = mine ? v : 0.0;
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (mine && (int)__lane_id() == leader) atomicAdd(&arr[key], s);
        active &= ~same;
    }
}

// Box, tile and cell-in-tile of global cell (x, y, z).
__device__ __forceinline__ int box_of_cell(const Geom &G, int x, int y, int z) {
    return G.coarse_box[(x / G.g[0]) + G.cg[0] * ((y / G.g[1]) + G.cg[1] * (z / G.g[2]))];
}

// Tile of box b holding the point (x, y, z) of that box, and the point's
// index inside the tile.
__device__ __forceinline__ void locate_in_box(const Geom &G, int b, int x, int y, int z, int &tile, int &local) {
    int lx = x - G.box_lo[3 * b], ly = y - G.box_lo[3 * b + 1], lz = z - G.box_lo[3 * b + 2];
    int tx = lx / G.T[0], ty = ly / G.T[1], tz = lz / G.T[2];
    tile = G.box_tile_off[b] + tx + G.box_nt[3 * b] * (ty + G.box_nt[3 * b + 1] * tz);
    local = (lx - tx * G.T[0]) + G.T[0] * ((ly - ty * G.T[1]) + G.T[1] * (lz - tz * G.T[2]));
}

}  // namespace pb
