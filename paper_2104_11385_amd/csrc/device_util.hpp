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

// Wraps a tile-relative coordinate r into [-h, n - h).  Only tiles on a
// periodic face need the wrap, so the test comes first.
__device__ __forceinline__ int wrap_rel(int r, int h, int n) {
    int t = r + h;
    if ((unsigned)t >= (unsigned)n) {
        t = t < 0 ? t + n : t - n;
        if ((unsigned)t >= (unsigned)n) t = wrap_any(t, n);
    }
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

// Lane moves inside 16-lane rows through DPP (every lane of the wave must be
// active): row_shr<S> gives lane i the value of lane i - S, row_shl<S> that
// of lane i + S; lanes whose source lies outside their row receive 0.
template <int S>
__device__ __forceinline__ int row_shr(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x110 + S, 0xF, 0xF, true);
}
template <int S>
__device__ __forceinline__ int row_shl(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x100 + S, 0xF, 0xF, true);
}
// Lane 16 r + 15 to the lanes of row r + 1 (rows 1-3; row 0 receives 0).
__device__ __forceinline__ int row_bcast15(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x142, 0xE, 0xF, false); }
template <int S>
__device__ __forceinline__ float row_shr(float v) {
    return __int_as_float(row_shr<S>(__float_as_int(v)));
}
template <int S>
__device__ __forceinline__ double row_shr(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = row_shr<S>((int)b), hi = row_shr<S>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double row_bcast15(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = row_bcast15((int)b), hi = row_bcast15((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Segments of equal keys in a 16-lane row (contiguous runs, keys never 0):
// m[j] = 1 when lanes i - 2^j .. i all hold lane i's key, else 0.
// A run that crosses one row boundary, into a row that it does not both fill
// and leave, is then summed across it: the lanes of the run's part in the
// later row add the sum at the earlier row's last lane (m[4] = 1), and that
// lane stops being a leader, so that the two rows' leaders of one run do not
// add to one LDS address in the same instruction.  A run over three rows or
// more keeps a leader per row (a correct sum in parts).
template <typename real>
struct RowRuns {
    real m[5];
    bool last;  // lane i holds the sum of its run (or of the run's part in its row)
    __device__ __forceinline__ void set(int key) {
        const int lane = (int)__lane_id(), row = lane >> 4, col = lane & 15;
        // key of the lane before, across rows too (DPP wave_shr:1)
        const bool eq = __builtin_amdgcn_update_dpp(0, key, 0x138, 0xF, 0xF, false) == key;
        const unsigned long long E = __ballot(eq);
        int f1 = eq && col != 0;
        int f2 = f1 & row_shr<1>(f1);
        int f4 = f2 & row_shr<2>(f2);
        int f8 = f4 & row_shr<4>(f4);
        m[0] = (real)f1;
        m[1] = (real)f2;
        m[2] = (real)f4;
        m[3] = (real)f8;
        last = row_shl<1>(key) != key;
        // wave-uniform: lanes where a run starts inside a row, runs across
        // the boundaries after rows 0, 1, 2, and which of them are merged
        const unsigned long long brk = ~E & ~0x0001000100010001ull;
        const bool c0 = (E >> 16) & 1, c1 = (E >> 32) & 1, c2 = (E >> 48) & 1;
        const bool w1 = ((brk >> 16) & 0xFFFFull) == 0, w2 = ((brk >> 32) & 0xFFFFull) == 0;
        const unsigned G = ((c0 && !(w1 && c1)) ? 2u : 0u) | ((c1 && !(w2 && c2)) ? 4u : 0u) | (c2 ? 8u : 0u);
        // the lane lies in the first run of its row: no run starts in its
        // row before it, and it starts none itself
        const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(brk >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)brk, 0u));
        const int r1 = __popcll(brk & 0xFFFFull), r2 = __popcll(brk & 0xFFFFFFFFull), r3 = __popcll(brk & 0xFFFFFFFFFFFFull);
        const int rowbase = row == 0 ? 0 : (row == 1 ? r1 : (row == 2 ? r2 : r3));
        const bool initial = below == rowbase && (eq || col == 0);
        m[4] = (real)(((G >> row) & 1u) && initial);
        last = last && !(col == 15 && ((G >> (row + 1)) & 1u));
    }
    // Inclusive segmented sum: the last lane of each run receives the run's
    // sum inside the row (Hillis-Steele steps 1, 2, 4, 8), then across one
    // row boundary.
    __device__ __forceinline__ real sum(real v) const {
        v = fma(row_shr<1>(v), m[0], v);
        v = fma(row_shr<2>(v), m[1], v);
        v = fma(row_shr<4>(v), m[2], v);
        v = fma(row_shr<8>(v), m[3], v);
        v = fma(row_bcast15(v), m[4], v);
        return v;
    }
    // The same sum of N single-precision values, one v_fmac_f32 with a DPP
    // source per value and step (v += m * v[lane - S]; lanes whose source
    // lies outside the row read 0).  The compiler does not fold its own DPP
    // moves into fmac, which would take two instructions per step.
    template <int N>
    __device__ __forceinline__ void sum_n(float (&v)[N]) const;
};

// Each statement starts with two wait states: a DPP read of a VGPR written
// by the instruction just before it needs them.  CTL is the whole DPP
// control (lane pattern and masks).
#define PB_FMAC_STEP6(CTL, v, k, m)                                                        \
    asm volatile("s_nop 1\n\t"                                                            \
                 "v_fmac_f32_dpp %0, %0, %6 " CTL "\n\t"                                   \
                 "v_fmac_f32_dpp %1, %1, %6 " CTL "\n\t"                                   \
                 "v_fmac_f32_dpp %2, %2, %6 " CTL "\n\t"                                   \
                 "v_fmac_f32_dpp %3, %3, %6 " CTL "\n\t"                                   \
                 "v_fmac_f32_dpp %4, %4, %6 " CTL "\n\t"                                   \
                 "v_fmac_f32_dpp %5, %5, %6 " CTL                                           \
                 : "+v"(v[k]), "+v"(v[k + 1]), "+v"(v[k + 2]), "+v"(v[k + 3]), "+v"(v[k + 4]),   \
                   "+v"(v[k + 5])                                                           \
                 : "v"(m))
#define PB_FMAC_STEP2(CTL, v, k, m)                                                        \
    asm volatile("s_nop 1\n\t"                                                            \
                 "v_fmac_f32_dpp %0, %0, %2 " CTL "\n\t"                                   \
                 "v_fmac_f32_dpp %1, %1, %2 " CTL                                           \
                 : "+v"(v[k]), "+v"(v[k + 1])                                               \
                 : "v"(m))
#define PB_ROW_SHR(S) "row_shr:" #S " row_mask:0xf bank_mask:0xf bound_ctrl:1"

template <>
template <int N>
__device__ __forceinline__ void RowRuns<float>::sum_n(float (&v)[N]) const {
    static_assert(N % 2 == 0, "sum_n takes an even count");
#define PB_FMAC_ALL(SH, mm)                                                                \
    {                                                                                      \
        int k = 0;                                                                         \
        _Pragma("unroll") for (; k + 6 <= N; k += 6) PB_FMAC_STEP6(SH, v, k, mm);          \
        _Pragma("unroll") for (; k + 2 <= N; k += 2) PB_FMAC_STEP2(SH, v, k, mm);          \
    }
    PB_FMAC_ALL(PB_ROW_SHR(1), m[0]);
    PB_FMAC_ALL(PB_ROW_SHR(2), m[1]);
    PB_FMAC_ALL(PB_ROW_SHR(4), m[2]);
    PB_FMAC_ALL(PB_ROW_SHR(8), m[3]);
    // rows 1-3 take lane 15 of the row before; row 0 is not written
    PB_FMAC_ALL("row_bcast:15 row_mask:0xe bank_mask:0xf", m[4]);
#undef PB_FMAC_ALL
}
#undef PB_FMAC_STEP6
#undef PB_FMAC_STEP2
#undef PB_ROW_SHR

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
