// gfx950 kernels of the PIC step: on-device particle loader, tile sort,
// gather-push-deposit with in-kernel per-box clock costs, Yee update, and
// the per-box counts and features used for load balancing.
//
// Numerical methods (the paper names the PIC scheme only in words, Sec. 2.1):
//   shapes   centred B-splines of order 1 or 2;
//   gather   each component interpolated at its own Yee stagger with the same
//            order-m spline;
//   push     relativistic Boris rotation (Boris 1970; Birdsall & Langdon);
//   deposit  Esirkepov (2001) charge-conserving density decomposition;
//   fields   Yee (1966): B half step, E full step with -J, B half step.
// Per-box costs follow Sec. 2.2 and Fig. 2a: a device clock is read around
// the compute-intensive work, summed on chip, then added once per block to a
// global per-box counter.
#include "kernels.hpp"

#include <hip/hip_runtime.h>

namespace pb {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

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
__device__ int block_excl_scan(int v, int *sh, int &total) {
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
__device__ void wave_count_add(unsigned long long *arr, int key) {
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

__device__ void wave_sum_add(double *arr, int key, double v) {
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

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and the particle loader
// ---------------------------------------------------------------------------

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

template <typename real>
__global__ void k_load(Particles<real> P, LoadArgs a) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    int cx, cy, cz;
    double w;
    if (a.mode == 1) {
        int64_t cellrank = p / a.ppc;
        cx = a.rlo[0] + (int)(cellrank % a.rext[0]);
        int64_t q = cellrank / a.rext[0];
        cy = a.rlo[1] + (int)(q % a.rext[1]);
        cz = a.rlo[2] + (int)(q / a.rext[1]);
        w = a.density / (double)a.ppc;
    } else {
        // box b with base[b] <= p < base[b+1]
        int lo = 0, hi = a.nb;  // base has nb+1 entries
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (a.box_base[mid] <= p) lo = mid;
            else hi = mid;
        }
        int b = lo;
        int ppc = a.box_ppc[b];
        int64_t local = (p - a.box_base[b]) / ppc;
        const int *bx = a.boxes6 + 6 * b;
        int ex = bx[3] - bx[0], ey = bx[4] - bx[1];
        cx = bx[0] + (int)(local % ex);
        cy = bx[1] + (int)((local / ex) % ey);
        cz = bx[2] + (int)(local / ((int64_t)ex * ey));
        w = a.density / (double)ppc;
    }
    uint32_t lo32 = (uint32_t)(uint64_t)p, hi32 = (uint32_t)((uint64_t)p >> 32);
    uint32_t r0[4] = {lo32, hi32, 0u, 0u}, r1[4] = {lo32, hi32, 1u, 0u};
    philox4x32_10(r0, a.k0, a.k1);
    philox4x32_10(r1, a.k0, a.k1);
    const double s24 = 1.0 / 16777216.0;
    double U0 = (double)(r0[0] >> 8) * s24, U1 = (double)(r0[1] >> 8) * s24, U2 = (double)(r0[2] >> 8) * s24;
    double ga = ((double)(r0[3] >> 8) + 1.0) * s24, gb = (double)(r1[0] >> 8) * s24;
    double gc = ((double)(r1[1] >> 8) + 1.0) * s24, ge = (double)(r1[2] >> 8) * s24;
    const double twopi = 6.283185307179586476925286766559;
    double ra = sqrt(-2.0 * log(ga)), rc = sqrt(-2.0 * log(gc));
    double n0 = ra * cos(twopi * gb), n1 = ra * sin(twopi * gb), n2 = rc * cos(twopi * ge);
    int64_t d = a.out_base + p;
    P.cell[d] = pack_cell(cx, cy, cz);
    P.f[0][d] = (real)U0;
    P.f[1][d] = (real)U1;
    P.f[2][d] = (real)U2;
    P.u[0][d] = (real)(a.uth[0] * n0 + a.udrift[0]);
    P.u[1][d] = (real)(a.uth[1] * n1 + a.udrift[1]);
    P.u[2][d] = (real)(a.uth[2] * n2 + a.udrift[2]);
    P.w[d] = (real)w;
    P.id[d] = p;
    P.sp[d] = (uint8_t)a.species;
}

// ---------------------------------------------------------------------------
// Tile sort.  Output order: by (tile, species), and inside a (tile, species)
// segment by (rank of the particle within its cell, cell).  Consecutive
// particles then sit in distinct cells, so the lanes of a wave deposit into
// distinct LDS addresses.  A particle belongs to the box of its cell (that
// box's timer pays for it, as the box counts say); inside the box, quadratic
// shapes use the nearest node as the "cell", which fixes the start of the
// deposit window and centres the tile's halo margin.  A node on the box's
// upper face falls back to the cell in that dimension.
// ---------------------------------------------------------------------------

template <typename real>
__device__ __forceinline__ void sort_point(const Particles<real> &P, const Geom &G, int p, int &b, int &x, int &y,
                                           int &z) {
    unpack_cell(P.cell[p], x, y, z);
    b = box_of_cell(G, x, y, z);
    if (G.order == 2) {
        const int *lo = G.box_lo + 3 * b, *nt = G.box_nt + 3 * b;
        x += (P.f[0][p] >= (real)0.5) && (x + 1 < lo[0] + nt[0] * G.T[0]);
        y += (P.f[1][p] >= (real)0.5) && (y + 1 < lo[1] + nt[1] * G.T[1]);
        z += (P.f[2][p] >= (real)0.5) && (z + 1 < lo[2] + nt[2] * G.T[2]);
    }
}

template <typename real>
__global__ void k_sort_key(Particles<real> P, int np, Geom G, uint32_t *cellcnt, uint32_t *key,
                           uint32_t *rank) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    int x, y, z, b, t, l;
    sort_point(P, G, p, b, x, y, z);
    locate_in_box(G, b, x, y, z, t, l);
    uint32_t k = (uint32_t)((t * G.nsp + P.sp[p]) * G.Tvol + l);
    key[p] = k;
    rank[p] = atomicAdd(&cellcnt[k], 1u);
}

__global__ void k_sort_seg(const uint32_t *cellcnt, uint32_t *cellstart, int *segtot, int Tvol) {
    __shared__ int sh[17];
    int ts = blockIdx.x;
    int v = (int)cellcnt[(size_t)ts * Tvol + threadIdx.x];
    int tot;
    int ex = block_excl_scan(v, sh, tot);
    cellstart[(size_t)ts * Tvol + threadIdx.x] = (uint32_t)ex;
    if (threadIdx.x == 0) segtot[ts] = tot;
}

// Exclusive scan of n ints into out[0..n] (out[n] = total); one block.
__global__ void k_scan_single(const int *in, int *out, int n) {
    __shared__ int sh[17];
    int per = (n + blockDim.x - 1) / blockDim.x;
    int b = threadIdx.x * per, e = min(n, b + per);
    int s = 0;
    for (int i = b; i < e; ++i) s += in[i];
    int tot;
    int ex = block_excl_scan(s, sh, tot);
    for (int i = b; i < e; ++i) {
        out[i] = ex;
        ex += in[i];
    }
    if (threadIdx.x == 0) out[n] = tot;
}

// Multi-block exclusive scan in three launches: block sums, a scan of the
// sums, and block-local scans offset by them.  Blocks of 1024 elements.
__global__ void k_scan_bsum(const int *in, int n, int *bsum) {
    __shared__ int sh[17];
    int i = blockIdx.x * 1024 + threadIdx.x;
    int v = i < n ? in[i] : 0;
    int tot;
    (void)block_excl_scan(v, sh, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_apply(const int *in, int n, const int *boff, int *out) {
    __shared__ int sh[17];
    int i = blockIdx.x * 1024 + threadIdx.x;
    int v = i < n ? in[i] : 0;
    int tot;
    int ex = block_excl_scan(v, sh, tot);
    if (i < n) out[i] = ex + boff[blockIdx.x];
    if (i == n - 1) out[n] = ex + v + boff[blockIdx.x];
}

__global__ void k_sort_levels(const uint32_t *cellcnt, const uint32_t *cellstart, const int *segstart,
                              uint32_t *table, int Tvol) {
    __shared__ int sh[17];
    __shared__ int smax;
    int ts = blockIdx.x;
    int base = segstart[ts];
    if (segstart[ts + 1] == base) return;
    size_t ci = (size_t)ts * Tvol + threadIdx.x;
    int cnt = (int)cellcnt[ci];
    int cs = (int)cellstart[ci];
    if (threadIdx.x == 0) smax = 0;
    __syncthreads();
    atomicMax(&smax, cnt);
    __syncthreads();
    int maxc = smax;
    int lvl = 0;
    for (int k = 0; k < maxc; ++k) {
        int flag = cnt > k;
        int tot;
        int r = block_excl_scan(flag, sh, tot);
        if (flag) table[base + cs + k] = (uint32_t)(base + lvl + r);
        lvl += tot;
    }
}

template <typename real>
__global__ void k_sort_scatter(Particles<real> S, Particles<real> D, int np, const uint32_t *key,
                               const uint32_t *rank, const uint32_t *cellstart, const int *segstart,
                               const uint32_t *table, int Tvol) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    uint32_t k = key[p];
    int ts = (int)(k / (uint32_t)Tvol);
    int idx = segstart[ts] + (int)cellstart[k] + (int)rank[p];
    int d = (int)table[idx];
    D.cell[d] = S.cell[p];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        D.f[c][d] = S.f[c][p];
        D.u[c][d] = S.u[c][p];
    }
    D.w[d] = S.w[p];
    D.id[d] = S.id[p];
    D.sp[d] = S.sp[p];
}

// ---------------------------------------------------------------------------
// Work queue for the persistent kernel: tiles cut into chunks of at most
// `chunk` particles, ordered largest first (size classes).
// ---------------------------------------------------------------------------

__device__ __forceinline__ int size_class(int sz, int chunk, int ncls) {
    int c = (int)(((long long)(chunk - sz) * ncls) / chunk);
    return c < 0 ? 0 : (c >= ncls ? ncls - 1 : c);
}

// Sub-queue of tile t: contiguous tile ranges holding equal shares of the
// particles, one per XCD, so that neighbouring tiles share an L2.
__device__ __forceinline__ int sub_queue(const int *segstart, int t, int ntiles, int nsp) {
    long long tot = segstart[ntiles * nsp];
    if (tot <= 0) return 0;
    int x = (int)(((long long)segstart[t * nsp] * kSubQueues) / tot);
    return x < kSubQueues ? x : kSubQueues - 1;
}

__global__ void k_queue_count(const int *segstart, int ntiles, int nsp, int chunk, int ncls, int *cls_cnt) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int n = segstart[(t + 1) * nsp] - segstart[t * nsp];
    if (n == 0) return;
    int x = sub_queue(segstart, t, ntiles, nsp);
    int full = n / chunk, rem = n - full * chunk;
    if (full) atomicAdd(&cls_cnt[x * ncls], full);
    if (rem) atomicAdd(&cls_cnt[x * ncls + size_class(rem, chunk, ncls)], 1);
}

// Bucket offsets: sub-queue major, size class (largest first) minor.
__global__ void k_queue_scan(int *cls_cnt, int *cursor, int ncls, int *qbounds) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int acc = 0;
    for (int x = 0; x < kSubQueues; ++x) {
        qbounds[x] = acc;
        for (int c = 0; c < ncls; ++c) {
            cursor[x * ncls + c] = acc;
            acc += cls_cnt[x * ncls + c];
            cls_cnt[x * ncls + c] = 0;
        }
    }
    qbounds[kSubQueues] = acc;
}

__global__ void k_queue_fill(const int *segstart, int ntiles, int nsp, int chunk, int ncls, int *cursor,
                             int4 *queue) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int b = segstart[t * nsp], n = segstart[(t + 1) * nsp] - b;
    if (n == 0) return;
    int x = sub_queue(segstart, t, ntiles, nsp);
    int full = n / chunk, rem = n - full * chunk;
    if (full) {
        int pos = atomicAdd(&cursor[x * ncls], full);
        for (int j = 0; j < full; ++j) queue[pos + j] = make_int4(t, b + j * chunk, b + (j + 1) * chunk, 0);
    }
    if (rem) {
        int pos = atomicAdd(&cursor[x * ncls + size_class(rem, chunk, ncls)], 1);
        queue[pos] = make_int4(t, b + full * chunk, b + n, 0);
    }
}

__global__ void k_reset_heads(int *heads) {
    if (threadIdx.x < kSubQueues && blockIdx.x == 0) heads[threadIdx.x] = 0;
}

__global__ void k_set_int(int *p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

template <typename T>
__global__ void k_fill(T *a, T v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) a[i] = v;
}

// ---------------------------------------------------------------------------
// Gather - push - deposit
// ---------------------------------------------------------------------------

// Compile-time tile configuration.  Positions are referred to the particle's
// cell (order 1) or nearest node (order 2); the staged E/B window reaches
// RL_EB below and RH_EB above it, the J window RL_J / RH_J, plus the tile
// halo H on both sides.
template <typename real, int M, int TX, int TY, int TZ, int H>
struct Cfg {
    static constexpr int RL_EB = (M == 1) ? 1 : 2, RH_EB = (M == 3) ? 2 : 1;
    static constexpr int RL_J = (M == 1) ? 1 : 2, RH_J = (M == 3) ? 3 : 2;
    static constexpr int EX = TX + 2 * H + RL_EB + RH_EB;
    static constexpr int EY = TY + 2 * H + RL_EB + RH_EB;
    static constexpr int EZ = TZ + 2 * H + RL_EB + RH_EB;
    static constexpr int JX = TX + 2 * H + RL_J + RH_J;
    static constexpr int JY = TY + 2 * H + RL_J + RH_J;
    static constexpr int JZ = TZ + 2 * H + RL_J + RH_J;
    static constexpr int NEB = EX * EY * EZ;
    static constexpr int NJ = JX * JY * JZ;
    // J is accumulated in double: gfx950's LDS atomic add is fast for f64
    // (and integers) but an order of magnitude slower for f32.
    static constexpr size_t lds = (size_t)(6 * NEB) * sizeof(real) + (size_t)(3 * NJ) * sizeof(double);
    // per-thread slot of the deferred-deposit queue: d0[3], D[3], coef, rel
    static constexpr size_t qslot = 7 * sizeof(real) + sizeof(int);
};

// Shape factors of one dimension.  Inputs: d = offset from the reference
// (order 1: cell offset f in [0,1); order 2: node offset in [-1/2, 1/2)).
// Gather weights at integer nodes (wn, first node at offset bn) and at half
// nodes (wh, first half node at offset bh, dynamic).
template <typename real, int M>
struct GatherW {
    real wn[M + 1], wh[M + 1];
    int bh;
    // cubic B-spline weights of the nodes at -1, 0, 1, 2 from a point at
    // fraction t in [0, 1) of its cell
    __device__ __forceinline__ static void cubic(real t, real *w) {
        const real sixth = (real)(1.0 / 6.0), tt = (real)(2.0 / 3.0);
        real u = (real)1 - t;
        w[0] = sixth * u * u * u;
        w[1] = tt - t * t + (real)0.5 * t * t * t;
        w[2] = tt - u * u + (real)0.5 * u * u * u;
        w[3] = sixth * t * t * t;
    }
    __device__ __forceinline__ void set(real d) {
        if (M == 3) {
            // reference is the cell; d = offset in [0, 1)
            cubic(d, wn);
            bool up = d >= (real)0.5;
            cubic(up ? d - (real)0.5 : d + (real)0.5, wh);
            bh = up ? -1 : -2;
        } else if (M == 1) {
            wn[0] = (real)1 - d;
            wn[1] = d;
            bool up = d >= (real)0.5;
            real t = up ? d - (real)0.5 : d + (real)0.5;
            bh = up ? 0 : -1;
            wh[0] = (real)1 - t;
            wh[1] = t;
        } else {
            const real h = (real)0.5;
            wn[0] = h * (h - d) * (h - d);
            wn[1] = (real)0.75 - d * d;
            wn[2] = h * (h + d) * (h + d);
            bool up = d >= (real)0;
            real t = up ? d - h : d + h;
            bh = up ? -1 : -2;
            wh[0] = h * (h - t) * (h - t);
            wh[1] = (real)0.75 - t * t;
            wh[2] = h * (h + t) * (h + t);
        }
    }
};

// Esirkepov window of one dimension: (M+2) nodes starting at offset s from
// the reference; S0 = old shape, dS = new - old shape.  When the particle
// keeps its reference node the differences are formed from the
// displacement itself (no cancellation).
template <typename real, int M>
struct DepW {
    real S0[M + 2], dS[M + 2];
    int s;
    bool moved;  // the particle left its reference cell / node this step
    __device__ __forceinline__ void set(real d0, real D) {
        real d1 = d0 + D;
        if (M == 3) {
            // reference is the cell, d0 in [0, 1); nodes at offsets -1..2
            int k = (d1 >= (real)1) - (d1 < (real)0);
            real f1 = d1 - (real)k;
            bool km = k < 0, kp = k > 0;
            real o[4], n[4];
            GatherW<real, 3>::cubic(d0, o);
            GatherW<real, 3>::cubic(f1, n);
            // window of 5 nodes from offset s = min(0, k) - 1
            S0[0] = km ? (real)0 : o[0];
            S0[1] = km ? o[0] : o[1];
            S0[2] = km ? o[1] : o[2];
            S0[3] = km ? o[2] : o[3];
            S0[4] = km ? o[3] : (real)0;
            real s1[5];
            s1[0] = kp ? (real)0 : n[0];
            s1[1] = kp ? n[0] : n[1];
            s1[2] = kp ? n[1] : n[2];
            s1[3] = kp ? n[2] : n[3];
            s1[4] = kp ? n[3] : (real)0;
#pragma unroll
            for (int a = 0; a < 5; ++a) dS[a] = s1[a] - S0[a];
            if (k == 0) {
                // differences formed from the displacement D = d1 - d0:
                // with Q(a, b) = a^2 + ab + b^2 and g = 1 - d,
                //   node -1: -D Q(g0, g1) / 6        node 2: D Q(d0, d1) / 6
                //   node  0: -D (d0 + d1) + D Q(d0, d1) / 2
                //   node  1:  D (g0 + g1) - D Q(g0, g1) / 2
                const real sixth = (real)(1.0 / 6.0), h = (real)0.5;
                real g0 = (real)1 - d0, g1 = (real)1 - d1;
                real qf = d0 * d0 + d0 * d1 + d1 * d1, qg = g0 * g0 + g0 * g1 + g1 * g1;
                dS[0] = -D * sixth * qg;
                dS[1] = -D * (d0 + d1) + h * D * qf;
                dS[2] = D * (g0 + g1) - h * D * qg;
                dS[3] = D * sixth * qf;
                dS[4] = (real)0;
            }
            s = km ? -2 : -1;
            moved = k != 0;
        } else if (M == 1) {
            int k = (d1 >= (real)1) - (d1 < (real)0);
            real f1 = d1 - (real)k;
            bool km = k < 0, kp = k > 0;
            real a0 = (real)1 - d0, b0 = d0;
            real a1 = (real)1 - f1, b1 = f1;
            S0[0] = km ? (real)0 : a0;
            S0[1] = km ? a0 : b0;
            S0[2] = km ? b0 : (real)0;
            real s10 = kp ? (real)0 : a1;
            real s11 = kp ? a1 : b1;
            real s12 = kp ? b1 : (real)0;
            dS[0] = s10 - S0[0];
            dS[1] = s11 - S0[1];
            dS[2] = s12 - S0[2];
            if (k == 0) {
                dS[0] = -D;
                dS[1] = D;
                dS[2] = (real)0;
            }
            s = km ? -1 : 0;
            moved = k != 0;
        } else {
            const real h = (real)0.5;
            int k = (d1 >= h) - (d1 < -h);
            real e = d1 - (real)k;
            bool km = k < 0, kp = k > 0;
            real A0 = h * (h - d0) * (h - d0), B0 = (real)0.75 - d0 * d0, C0 = h * (h + d0) * (h + d0);
            real A1 = h * (h - e) * (h - e), B1 = (real)0.75 - e * e, C1 = h * (h + e) * (h + e);
            S0[0] = km ? (real)0 : A0;
            S0[1] = km ? A0 : B0;
            S0[2] = km ? B0 : C0;
            S0[3] = km ? C0 : (real)0;
            real s1[4];
            s1[0] = kp ? (real)0 : A1;
            s1[1] = kp ? A1 : B1;
            s1[2] = kp ? B1 : C1;
            s1[3] = kp ? C1 : (real)0;
#pragma unroll
            for (int a = 0; a < 4; ++a) dS[a] = s1[a] - S0[a];
            if (k == 0) {
                real sg = d0 + d1;
                dS[0] = -h * D * ((real)1 - sg);
                dS[1] = -D * sg;
                dS[2] = h * D * ((real)1 + sg);
                dS[3] = (real)0;
            }
            s = km ? -2 : -1;
            moved = k != 0;
        }
    }
    // The particle keeps its reference (cell or node): window of M+1 nodes
    // from offset s, differences from the displacement (no cancellation).
    __device__ __forceinline__ void set_kept(real d0, real D) {
        real d1 = d0 + D;
        if (M == 3) {
            const real sixth = (real)(1.0 / 6.0), tt = (real)(2.0 / 3.0), h = (real)0.5;
            real u = (real)1 - d0;
            S0[0] = sixth * u * u * u;
            S0[1] = tt - d0 * d0 + h * d0 * d0 * d0;
            S0[2] = tt - u * u + h * u * u * u;
            S0[3] = sixth * d0 * d0 * d0;
            real g0 = (real)1 - d0, g1 = (real)1 - d1;
            real qf = d0 * d0 + d0 * d1 + d1 * d1, qg = g0 * g0 + g0 * g1 + g1 * g1;
            dS[0] = -D * sixth * qg;
            dS[1] = -D * (d0 + d1) + h * D * qf;
            dS[2] = D * (g0 + g1) - h * D * qg;
            dS[3] = D * sixth * qf;
            s = -1;
        } else if (M == 1) {
            S0[0] = (real)1 - d0;
            S0[1] = d0;
            dS[0] = -D;
            dS[1] = D;
            s = 0;
        } else {
            const real h = (real)0.5;
            S0[0] = h * (h - d0) * (h - d0);
            S0[1] = (real)0.75 - d0 * d0;
            S0[2] = h * (h + d0) * (h + d0);
            real sg = d0 + d1;
            dS[0] = -h * D * ((real)1 - sg);
            dS[1] = -D * sg;
            dS[2] = h * D * ((real)1 + sg);
            s = -1;
        }
        moved = false;
    }
};

// Whether a displacement D from reference offset d0 leaves the reference
// cell (orders 1, 3: d0 in [0, 1)) or node (order 2: d0 in [-1/2, 1/2)).
template <typename real, int M>
__device__ __forceinline__ bool leaves_ref(real d0, real D) {
    real d1 = d0 + D;
    if (M == 2) return d1 >= (real)0.5 || d1 < (real)-0.5;
    return d1 >= (real)1 || d1 < (real)0;
}

// Interpolates the six field components from an accessor F(comp, i, j, k)
// where (i,j,k) are offsets from the particle's reference.
template <typename real, int M, typename Acc>
__device__ __forceinline__ void gather6(const Acc &F, const GatherW<real, M> W[3], real EB[6]) {
    const int bn = (M == 1) ? 0 : -1;
    // stagger pattern per component: 1 = half node along that axis
    const int pat[6][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {0, 1, 1}, {1, 0, 1}, {1, 1, 0}};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const real *wx = pat[c][0] ? W[0].wh : W[0].wn;
        const real *wy = pat[c][1] ? W[1].wh : W[1].wn;
        const real *wz = pat[c][2] ? W[2].wh : W[2].wn;
        int ox = pat[c][0] ? W[0].bh : bn;
        int oy = pat[c][1] ? W[1].bh : bn;
        int oz = pat[c][2] ? W[2].bh : bn;
        real acc = (real)0;
        F.begin(c, ox, oy, oz);
#pragma unroll
        for (int k = 0; k <= M; ++k) {
            real ay = (real)0;
#pragma unroll
            for (int j = 0; j <= M; ++j) {
                real ax = (real)0;
#pragma unroll
                for (int i = 0; i <= M; ++i) ax += wx[i] * F.tap(i, j, k);
                ay += wy[j] * ax;
            }
            acc += wz[k] * ay;
        }
        EB[c] = acc;
    }
}

// Deposits the Esirkepov current through an accessor J.add(comp, a, b, c, v)
// with (a,b,c) offsets inside the window.  L = M + 2 is the general window;
// a particle that keeps its reference node in every dimension has all its
// weight on the first M + 1 nodes and uses L = M + 1 (the last running sum
// along each axis is then zero by construction and is not deposited).
// The transverse factor of the density decomposition,
//   S0_u S0_v + (dS_u S0_v + S0_u dS_v) / 2 + dS_u dS_v / 3,
// equals A_u S0_v + B_u dS_v with A = S0 + dS/2 and B = S0/2 + dS/3; the
// charge factor -q w / dt is folded into A and B.
template <typename real, int M, int L, typename Acc>
__device__ __forceinline__ void deposit3(Acc &J, const DepW<real, M> W[3], real coef) {
    const real h = (real)0.5, third = (real)(1.0 / 3.0);
    real Ax[L], Bx[L], Ay[L], By[L];
#pragma unroll
    for (int a = 0; a < L; ++a) {
        Ax[a] = coef * (W[0].S0[a] + h * W[0].dS[a]);
        Bx[a] = coef * (h * W[0].S0[a] + third * W[0].dS[a]);
        Ay[a] = coef * (W[1].S0[a] + h * W[1].dS[a]);
        By[a] = coef * (h * W[1].S0[a] + third * W[1].dS[a]);
    }
    J.begin(W[0].s, W[1].s, W[2].s);
    // Jx: running sum along x of dSx * (A_y S0_z + B_y dS_z)
#pragma unroll
    for (int c = 0; c < L; ++c)
#pragma unroll
        for (int b = 0; b < L; ++b) {
            real in = Ay[b] * W[2].S0[c] + By[b] * W[2].dS[c];
            real acc = (real)0;
#pragma unroll
            for (int a = 0; a < L - 1; ++a) {
                acc += W[0].dS[a] * in;
                J.add(0, a, b, c, acc);
            }
        }
    // Jy: running sum along y of dSy * (A_x S0_z + B_x dS_z)
#pragma unroll
    for (int c = 0; c < L; ++c)
#pragma unroll
        for (int a = 0; a < L; ++a) {
            real in = Ax[a] * W[2].S0[c] + Bx[a] * W[2].dS[c];
            real acc = (real)0;
#pragma unroll
            for (int b = 0; b < L - 1; ++b) {
                acc += W[1].dS[b] * in;
                J.add(1, a, b, c, acc);
            }
        }
    // Jz: running sum along z of dSz * (A_x S0_y + B_x dS_y)
#pragma unroll
    for (int b = 0; b < L; ++b)
#pragma unroll
        for (int a = 0; a < L; ++a) {
            real in = Ax[a] * W[1].S0[b] + Bx[a] * W[1].dS[b];
            real acc = (real)0;
#pragma unroll
            for (int c = 0; c < L - 1; ++c) {
                acc += W[2].dS[c] * in;
                J.add(2, a, b, c, acc);
            }
        }
}

// Accessors: staged LDS windows (compile-time strides) ...
template <typename real, typename C>
struct LdsEB {
    const real *s;
    int ref;  // linear LDS index of the reference node (component 0)
    mutable int base;
    __device__ __forceinline__ void begin(int c, int ox, int oy, int oz) const {
        base = c * C::NEB + ref + ox + C::EX * (oy + C::EY * oz);
    }
    __device__ __forceinline__ real tap(int i, int j, int k) const {
        return s[base + i + C::EX * (j + C::EY * k)];
    }
};

template <typename real, typename C>
struct LdsJ {
    double *s;
    int ref;
    int base;
    __device__ __forceinline__ void begin(int sx, int sy, int sz) {
        base = ref + sx + C::JX * (sy + C::JY * sz);
    }
    __device__ __forceinline__ void add(int comp, int a, int b, int c, real v) {
        atomic_add_lds(&s[comp * C::NJ + base + a + C::JX * (b + C::JY * c)], (double)v);
    }
};

// ... and global arrays with periodic wrap (particles beyond the halo).
template <typename real>
struct GlobEB {
    const real *const *EB;
    int n[3], r[3];
    mutable const real *arr;
    mutable int ix[4], iy[4], iz[4];
    __device__ __forceinline__ void begin(int c, int ox, int oy, int oz) const {
        arr = EB[c];
        for (int q = 0; q < 4; ++q) {
            ix[q] = wrap_any(r[0] + ox + q, n[0]);
            iy[q] = wrap_any(r[1] + oy + q, n[1]);
            iz[q] = wrap_any(r[2] + oz + q, n[2]);
        }
    }
    __device__ __forceinline__ real tap(int i, int j, int k) const {
        return arr[ix[i] + (size_t)n[0] * (iy[j] + (size_t)n[1] * iz[k])];
    }
};

template <typename real>
struct GlobJ {
    real *const *J;
    int n[3], r[3];
    int ix[5], iy[5], iz[5];
    __device__ __forceinline__ void begin(int sx, int sy, int sz) {
        for (int q = 0; q < 5; ++q) {
            ix[q] = wrap_any(r[0] + sx + q, n[0]);
            iy[q] = wrap_any(r[1] + sy + q, n[1]);
            iz[q] = wrap_any(r[2] + sz + q, n[2]);
        }
    }
    __device__ __forceinline__ void add(int comp, int a, int b, int c, real v) {
        atomic_add_global(&J[comp][ix[a] + (size_t)n[0] * (iy[b] + (size_t)n[1] * iz[c])], v);
    }
};

// One particle's state as loaded from HBM.
template <typename real>
struct PState {
    uint32_t cell;
    real f[3], u[3], w;
    __device__ __forceinline__ void load(const Particles<real> &P, int p) {
        cell = P.cell[p];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            f[d] = P.f[d][p];
            u[d] = P.u[d][p];
        }
        w = P.w[p];
    }
};

// A particle that changed its reference node inside the staged window: its
// wider deposit waits in the wave's queue so that it runs with the other
// queued particles on full waves rather than on otherwise idle lanes.
template <typename real>
struct Deferred {
    bool want;
    int rel;          // packed window-relative reference node, +8 per byte
    real d0[3], D[3], coef;
};

template <typename real, int M, int TX, int TY, int TZ, int H>
__device__ __forceinline__ void push_particle(const GpdArgs<real> &A, int p, const PState<real> &ps,
                                              const TileDesc &td, real hq, real cq, const real *sEB, double *sJ,
                                              unsigned &nslow, Deferred<real> &df) {
    using C = Cfg<real, M, TX, TY, TZ, H>;
    int c[3];
    unpack_cell(ps.cell, c[0], c[1], c[2]);
    real f[3] = {ps.f[0], ps.f[1], ps.f[2]};
    real u[3] = {ps.u[0], ps.u[1], ps.u[2]};
    real w = ps.w;

    // reference point: cell (order 1) or nearest node (order 2)
    int ref[3];
    real d0[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (M == 2) {
            bool up = f[d] >= (real)0.5;
            ref[d] = c[d] + (up ? 1 : 0);
            d0[d] = up ? f[d] - (real)1 : f[d];
        } else {
            ref[d] = c[d];
            d0[d] = f[d];
        }
    }
    const int T[3] = {TX, TY, TZ};
    const int org[3] = {td.x0, td.y0, td.z0};
    int rel[3];
    bool fast = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        rel[d] = wrap_rel(ref[d] - org[d], H, A.n[d]);
        fast = fast && rel[d] <= T[d] + H - 1;
    }

    GatherW<real, M> GW[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) GW[d].set(d0[d]);
    real EB[6];
    if (fast) {
        LdsEB<real, C> acc{sEB, (rel[0] + H + C::RL_EB) + C::EX * ((rel[1] + H + C::RL_EB) + C::EY * (rel[2] + H + C::RL_EB)), 0};
        gather6<real, M>(acc, GW, EB);
    } else {
        GlobEB<real> acc;
        acc.EB = A.EB;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            acc.n[d] = A.n[d];
            acc.r[d] = ref[d];
        }
        gather6<real, M>(acc, GW, EB);
        ++nslow;
    }
    // the arrays hold B minus its uniform external part (whose curl is zero)
    EB[3] += A.bext[0];
    EB[4] += A.bext[1];
    EB[5] += A.bext[2];

    // relativistic Boris rotation
    real um[3] = {u[0] + hq * EB[0], u[1] + hq * EB[1], u[2] + hq * EB[2]};
    real ig = rsqrt_r((real)1 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    real t[3] = {hq * EB[3] * ig, hq * EB[4] * ig, hq * EB[5] * ig};
    real t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    real sf = (real)2 * rcp_r((real)1 + t2);
    real s[3] = {sf * t[0], sf * t[1], sf * t[2]};
    real up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]), um[1] + (um[2] * t[0] - um[0] * t[2]),
                  um[2] + (um[0] * t[1] - um[1] * t[0])};
    u[0] = um[0] + (up[1] * s[2] - up[2] * s[1]) + hq * EB[0];
    u[1] = um[1] + (up[2] * s[0] - up[0] * s[2]) + hq * EB[1];
    u[2] = um[2] + (up[0] * s[1] - up[1] * s[0]) + hq * EB[2];
    real gi = rsqrt_r((real)1 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    real D[3] = {A.dt * u[0] * gi, A.dt * u[1] * gi, A.dt * u[2] * gi};

    // Esirkepov deposit
    real coef = cq * w;
    bool moved = leaves_ref<real, M>(d0[0], D[0]) || leaves_ref<real, M>(d0[1], D[1]) ||
                 leaves_ref<real, M>(d0[2], D[2]);
    if (fast) {
        if (moved) {
            df.want = true;
            df.rel = (rel[0] + 8) | ((rel[1] + 8) << 8) | ((rel[2] + 8) << 16);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                df.d0[d] = d0[d];
                df.D[d] = D[d];
            }
            df.coef = coef;
        } else {
            DepW<real, M> DW[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) DW[d].set_kept(d0[d], D[d]);
            LdsJ<real, C> acc{sJ, (rel[0] + H + C::RL_J) + C::JX * ((rel[1] + H + C::RL_J) + C::JY * (rel[2] + H + C::RL_J)), 0};
            deposit3<real, M, M + 1>(acc, DW, coef);
        }
    } else {
        DepW<real, M> DW[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) DW[d].set(d0[d], D[d]);
        GlobJ<real> acc;
        acc.J = A.J;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            acc.n[d] = A.n[d];
            acc.r[d] = ref[d];
        }
        deposit3<real, M, M + 2>(acc, DW, coef);
    }

    // new canonical position: cell + offset in [0, 1), periodic wrap
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        real x = f[d] + D[d];
        int k = 0;
        if (x < (real)0) {
            x += (real)1;
            k = -1;
            if (x >= (real)1) {
                x = (real)0;
                k = 0;
            }
        } else if (x >= (real)1) {
            x -= (real)1;
            k = 1;
        }
        int cc = c[d] + k;
        if (cc < 0) cc += A.n[d];
        else if (cc >= A.n[d]) cc -= A.n[d];
        c[d] = cc;
        f[d] = x;
    }
    A.P.cell[p] = pack_cell(c[0], c[1], c[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        A.P.f[d][p] = f[d];
        A.P.u[d][p] = u[d];
    }
}

// Deposits queue entry s (word k of slot s lives at q[k * stride + s]).
template <typename real, int M, int TX, int TY, int TZ, int H>
__device__ __forceinline__ void deposit_queued(const real *qr, const int *qi, int stride, int s, double *sJ) {
    using C = Cfg<real, M, TX, TY, TZ, H>;
    {
        const int pk = qi[s];
        const int r0 = (pk & 255) - 8, r1 = ((pk >> 8) & 255) - 8, r2 = ((pk >> 16) & 255) - 8;
        DepW<real, M> DW[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) DW[d].set(qr[d * stride + s], qr[(3 + d) * stride + s]);
        const real coef = qr[6 * stride + s];
        LdsJ<real, C> acc{sJ, (r0 + H + C::RL_J) + C::JX * ((r1 + H + C::RL_J) + C::JY * (r2 + H + C::RL_J)), 0};
        deposit3<real, M, M + 2>(acc, DW, coef);
    }
}

// Deposits the first n entries of a wave's queue, one per lane.
template <typename real, int M, int TX, int TY, int TZ, int H>
__device__ __forceinline__ void drain_queue(const real *qr, const int *qi, int stride, int slot0, int n, int lane,
                                            double *sJ) {
    if (lane < n) deposit_queued<real, M, TX, TY, TZ, H>(qr, qi, stride, slot0 + lane, sJ);
}

template <typename real, int M, int TX, int TY, int TZ, int H>
__global__ __launch_bounds__(512) void k_gpd(GpdArgs<real> A) {
    using C = Cfg<real, M, TX, TY, TZ, H>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    real *sEB = reinterpret_cast<real *>(smem_raw);
    double *sJ = reinterpret_cast<double *>(smem_raw + (size_t)6 * C::NEB * sizeof(real));
    real *qr = reinterpret_cast<real *>(smem_raw + C::lds);           // [7][blockDim.x]
    int *qi = reinterpret_cast<int *>(qr + 7 * blockDim.x);          // [blockDim.x]
    __shared__ unsigned long long sCyc, sRtc;
    __shared__ unsigned int sSlow;
    __shared__ int sItem[3];
    __shared__ int sQn[8];  // queue lengths of the block's waves at the end of an item
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int nsp = A.nsp;
    const int home = blockIdx.x % kSubQueues;  // blocks are dealt round-robin over the XCDs
    // windows reach at most JX cells; one conditional wrap suffices unless the
    // domain is smaller than a window
    const bool small = A.n[0] < C::JX || A.n[1] < C::JY || A.n[2] < C::JZ;
    int sq = 0;                                // sub-queues already found empty (thread 0)

    for (int iter = 0;; ++iter) {
        int tile, pbeg, pend;
        if (A.mode == MODE_PERSISTENT) {
            // own XCD's sub-queue first, then steal from the others
            if (tid == 0) {
                sItem[0] = -1;
                for (; sq < kSubQueues; ++sq) {
                    int x = (home + sq) % kSubQueues;
                    int lo = A.queue_bounds[x], hi = A.queue_bounds[x + 1];
                    if (hi <= lo) continue;
                    int q = atomicAdd(&A.queue_head[x], 1);
                    if (lo + q < hi) {
                        int4 it = A.queue[lo + q];
                        sItem[0] = it.x;
                        sItem[1] = it.y;
                        sItem[2] = it.z;
                        break;
                    }
                }
            }
            __syncthreads();
            tile = sItem[0];
            pbeg = sItem[1];
            pend = sItem[2];
            if (tile < 0) break;
        } else {
            if (iter > 0) break;
            tile = A.tile_base + blockIdx.x;
            if (A.species_only >= 0) {
                pbeg = A.segstart[tile * nsp + A.species_only];
                pend = A.segstart[tile * nsp + A.species_only + 1];
            } else {
                pbeg = A.segstart[tile * nsp];
                pend = A.segstart[(tile + 1) * nsp];
            }
            if (pbeg >= pend) break;
        }
        const TileDesc td = A.tiles[tile];

        // stage E and B of the tile window (one index computation serves the
        // six components; windows inside the domain need no wrap); clear the
        // J window
        {
            const int ox = td.x0 - H - C::RL_EB, oy = td.y0 - H - C::RL_EB, oz = td.z0 - H - C::RL_EB;
            const bool inside = ox >= 0 && oy >= 0 && oz >= 0 && ox + C::EX <= A.n[0] && oy + C::EY <= A.n[1] &&
                                oz + C::EZ <= A.n[2];
            const size_t sy = (size_t)A.n[0], sz = (size_t)A.n[0] * A.n[1];
            for (int i = tid; i < C::NEB; i += nthr) {
                int lx = i % C::EX;
                int r2 = i / C::EX;
                int ly = r2 % C::EY;
                int lz = r2 / C::EY;
                int gx = ox + lx, gy = oy + ly, gz = oz + lz;
                if (!inside) {
                    if (small) {
                        gx = wrap_any(gx, A.n[0]);
                        gy = wrap_any(gy, A.n[1]);
                        gz = wrap_any(gz, A.n[2]);
                    } else {
                        gx = wrap_near(gx, A.n[0]);
                        gy = wrap_near(gy, A.n[1]);
                        gz = wrap_near(gz, A.n[2]);
                    }
                }
                const size_t g = (size_t)gx + sy * gy + sz * gz;
                real v[6];
#pragma unroll
                for (int comp = 0; comp < 6; ++comp) v[comp] = A.EB[comp][g];
#pragma unroll
                for (int comp = 0; comp < 6; ++comp) sEB[comp * C::NEB + i] = v[comp];
            }
        }
        for (int i = tid; i < 3 * C::NJ; i += nthr) sJ[i] = 0.0;
        if (tid == 0) {
            sCyc = 0;
            sRtc = 0;
            sSlow = 0;
        }
        __syncthreads();

        unsigned long long c0 = clock64(), r0 = wall_clock64();
        unsigned nslow = 0;
        const int lane = tid & 63, qslot0 = tid & ~63;
        int qn = 0;  // entries in this wave's queue (wave-uniform)
        for (int s = 0; s < nsp; ++s) {
            if (A.mode == MODE_PER_BOX && s != A.species_only) continue;
            int sb = max(pbeg, A.segstart[tile * nsp + s]);
            int se = min(pend, A.segstart[tile * nsp + s + 1]);
            real hq = A.h[s], cq = A.coefq[s];
            // the next particle's loads are issued before this one is computed;
            // the trip count is the same for every lane of the block
            PState<real> cur;
            if (sb + tid < se) cur.load(A.P, sb + tid);
            for (int base = sb; base < se; base += nthr) {
                const int p = base + tid;
                PState<real> nxt;
                if (p + nthr < se) nxt.load(A.P, p + nthr);
                Deferred<real> df;
                df.want = false;
                if (p < se) push_particle<real, M, TX, TY, TZ, H>(A, p, cur, td, hq, cq, sEB, sJ, nslow, df);
                const unsigned long long mask = __ballot(df.want);
                if (mask) {
                    const int cnt = __popcll(mask);
                    if (qn + cnt > 64) {
                        drain_queue<real, M, TX, TY, TZ, H>(qr, qi, nthr, qslot0, qn, lane, sJ);
                        qn = 0;
                    }
                    if (df.want) {
                        const int s2 = qslot0 + qn + __popcll(mask & ((1ull << lane) - 1ull));
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            qr[d * nthr + s2] = df.d0[d];
                            qr[(3 + d) * nthr + s2] = df.D[d];
                        }
                        qr[6 * nthr + s2] = df.coef;
                        qi[s2] = df.rel;
                    }
                    qn += cnt;
                }
                cur = nxt;
            }
        }
        // the entries left in the waves' queues are deposited by the block
        // together, one per thread, instead of by each wave on its own
        if (lane == 0) sQn[tid >> 6] = qn;
        __syncthreads();
        {
            const int nw = nthr >> 6;
            int e = tid, w = 0;
            while (w < nw && e >= sQn[w]) e -= sQn[w++];
            if (w < nw) deposit_queued<real, M, TX, TY, TZ, H>(qr, qi, nthr, w * 64 + e, sJ);
        }
        unsigned long long c1 = clock64(), r1 = wall_clock64();
        if ((tid & 63) == 0) {
            atomicAdd(&sCyc, c1 - c0);
            atomicAdd(&sRtc, r1 - r0);
        }
        if (nslow) atomicAdd(&sSlow, nslow);
        __syncthreads();

        // flush the J window (nonzero entries only)
        {
            const int ox = td.x0 - H - C::RL_J, oy = td.y0 - H - C::RL_J, oz = td.z0 - H - C::RL_J;
            const bool inside = ox >= 0 && oy >= 0 && oz >= 0 && ox + C::JX <= A.n[0] && oy + C::JY <= A.n[1] &&
                                oz + C::JZ <= A.n[2];
            const size_t sy = (size_t)A.n[0], sz = (size_t)A.n[0] * A.n[1];
            for (int i = tid; i < C::NJ; i += nthr) {
                real v[3];
#pragma unroll
                for (int comp = 0; comp < 3; ++comp) v[comp] = (real)sJ[comp * C::NJ + i];
                if (v[0] == (real)0 && v[1] == (real)0 && v[2] == (real)0) continue;
                int lx = i % C::JX;
                int r2 = i / C::JX;
                int ly = r2 % C::JY;
                int lz = r2 / C::JY;
                int gx = ox + lx, gy = oy + ly, gz = oz + lz;
                if (!inside) {
                    if (small) {
                        gx = wrap_any(gx, A.n[0]);
                        gy = wrap_any(gy, A.n[1]);
                        gz = wrap_any(gz, A.n[2]);
                    } else {
                        gx = wrap_near(gx, A.n[0]);
                        gy = wrap_near(gy, A.n[1]);
                        gz = wrap_near(gz, A.n[2]);
                    }
                }
                const size_t g = (size_t)gx + sy * gy + sz * gz;
#pragma unroll
                for (int comp = 0; comp < 3; ++comp)
                    if (v[comp] != (real)0) atomic_add_global(&A.J[comp][g], v[comp]);
            }
        }
        if (tid == 0) {
            atomicAdd(&A.cycles[td.box], sCyc);
            atomicAdd(&A.rtc[td.box], sRtc);
            if (sSlow) atomicAdd(A.slow, sSlow);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Yee update in three streaming passes.  Threads own (x, y) columns and march
// along z, carrying the z neighbours in registers; x and y neighbours are
// read through the caches.
//   pass 1 (in place): B <- B^{n+1/2} = B^n - dt/2 curl E^n
//   pass 2: E^{n+1} = E^n + dt (curl B^{n+1/2} - J) into the other E buffer,
//           and the next step's J buffer cleared
//   pass 3: B^{n+1} = B^{n+1/2} - dt/2 curl E^{n+1} into the other B buffer
// Curl of E uses forward differences, curl of B backward ones (Yee cell).
// ---------------------------------------------------------------------------

constexpr int YSX = 64, YSY = 4, YSZ = 4;

struct YeeArgs {
    const void *E[3], *J[3];
    void *B[3];             // B^n in, B^{n+1/2} out (pass 1); B^{n+1/2} in (pass 2)
    void *Eo[3], *Bo[3], *Z[3];
    int n[3];
    double dt;
};

template <typename real>
__global__ __launch_bounds__(256) void k_yee_bhalf(YeeArgs a) {
    const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
    const int x = blockIdx.x * YSX + (threadIdx.x & (YSX - 1));
    const int y = blockIdx.y * YSY + (threadIdx.x / YSX);
    if (x >= nx || y >= ny) return;
    const int z0 = blockIdx.z * YSZ, z1 = min(nz, z0 + YSZ);
    const real hdt = (real)(0.5 * a.dt);
    const real *Ex = (const real *)a.E[0], *Ey = (const real *)a.E[1], *Ez = (const real *)a.E[2];
    real *Bx = (real *)a.B[0], *By = (real *)a.B[1], *Bz = (real *)a.B[2];
    const size_t sxy = (size_t)nx * ny;
    const int xp = x + 1 == nx ? 0 : x + 1, yp = y + 1 == ny ? 0 : y + 1;
    const size_t col = (size_t)x + (size_t)nx * y, colx = (size_t)xp + (size_t)nx * y,
                 coly = (size_t)x + (size_t)nx * yp;
    size_t g = col + sxy * z0;
    real ex = Ex[g], ey = Ey[g];
    for (int k = z0; k < z1; ++k) {
        const size_t gk = sxy * k, gn = sxy * (k + 1 == nz ? 0 : k + 1);
        const real exn = Ex[col + gn], eyn = Ey[col + gn];
        const real ez = Ez[col + gk];
        const real eyx = Ey[colx + gk], ezx = Ez[colx + gk];
        const real exy = Ex[coly + gk], ezy = Ez[coly + gk];
        const real cx = (ezy - ez) - (eyn - ey);
        const real cy = (exn - ex) - (ezx - ez);
        const real cz = (eyx - ey) - (exy - ex);
        g = col + gk;
        Bx[g] = Bx[g] - hdt * cx;
        By[g] = By[g] - hdt * cy;
        Bz[g] = Bz[g] - hdt * cz;
        ex = exn;
        ey = eyn;
    }
}

template <typename real>
__global__ __launch_bounds__(256) void k_yee_e(YeeArgs a) {
    const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
    const int x = blockIdx.x * YSX + (threadIdx.x & (YSX - 1));
    const int y = blockIdx.y * YSY + (threadIdx.x / YSX);
    if (x >= nx || y >= ny) return;
    const int z0 = blockIdx.z * YSZ, z1 = min(nz, z0 + YSZ);
    const real dt = (real)a.dt;
    const real *Ex = (const real *)a.E[0], *Ey = (const real *)a.E[1], *Ez = (const real *)a.E[2];
    const real *Jx = (const real *)a.J[0], *Jy = (const real *)a.J[1], *Jz = (const real *)a.J[2];
    const real *Hx = (const real *)a.B[0], *Hy = (const real *)a.B[1], *Hz = (const real *)a.B[2];
    const size_t sxy = (size_t)nx * ny;
    const int xm = x == 0 ? nx - 1 : x - 1, ym = y == 0 ? ny - 1 : y - 1;
    const size_t c0 = (size_t)x + (size_t)nx * y, cxm = (size_t)xm + (size_t)nx * y, cym = (size_t)x + (size_t)nx * ym;
    const size_t gm = sxy * (z0 == 0 ? nz - 1 : z0 - 1);
    real hx_m = Hx[c0 + gm], hy_m = Hy[c0 + gm];
    for (int k = z0; k < z1; ++k) {
        const size_t gk = sxy * k, g = c0 + gk;
        const real hx = Hx[g], hy = Hy[g], hz = Hz[g];
        const real hzym = Hz[cym + gk], hzxm = Hz[cxm + gk], hyxm = Hy[cxm + gk], hxym = Hx[cym + gk];
        ((real *)a.Eo[0])[g] = Ex[g] + dt * (((hz - hzym) - (hy - hy_m)) - Jx[g]);
        ((real *)a.Eo[1])[g] = Ey[g] + dt * (((hx - hx_m) - (hz - hzxm)) - Jy[g]);
        ((real *)a.Eo[2])[g] = Ez[g] + dt * (((hy - hyxm) - (hx - hxym)) - Jz[g]);
        ((real *)a.Z[0])[g] = (real)0;
        ((real *)a.Z[1])[g] = (real)0;
        ((real *)a.Z[2])[g] = (real)0;
        hx_m = hx;
        hy_m = hy;
    }
}

template <typename real>
__global__ __launch_bounds__(256) void k_yee_b2(YeeArgs a) {
    const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
    const int x = blockIdx.x * YSX + (threadIdx.x & (YSX - 1));
    const int y = blockIdx.y * YSY + (threadIdx.x / YSX);
    if (x >= nx || y >= ny) return;
    const int z0 = blockIdx.z * YSZ, z1 = min(nz, z0 + YSZ);
    const real hdt = (real)(0.5 * a.dt);
    const real *Ex = (const real *)a.Eo[0], *Ey = (const real *)a.Eo[1], *Ez = (const real *)a.Eo[2];
    const real *Hx = (const real *)a.B[0], *Hy = (const real *)a.B[1], *Hz = (const real *)a.B[2];
    const size_t sxy = (size_t)nx * ny;
    const int xp = x + 1 == nx ? 0 : x + 1, yp = y + 1 == ny ? 0 : y + 1;
    const size_t col = (size_t)x + (size_t)nx * y, colx = (size_t)xp + (size_t)nx * y,
                 coly = (size_t)x + (size_t)nx * yp;
    size_t g = col + sxy * z0;
    real ex = Ex[g], ey = Ey[g];
    for (int k = z0; k < z1; ++k) {
        const size_t gk = sxy * k, gn = sxy * (k + 1 == nz ? 0 : k + 1);
        const real exn = Ex[col + gn], eyn = Ey[col + gn];
        const real ez = Ez[col + gk];
        const real eyx = Ey[colx + gk], ezx = Ez[colx + gk];
        const real exy = Ex[coly + gk], ezy = Ez[coly + gk];
        g = col + gk;
        ((real *)a.Bo[0])[g] = Hx[g] - hdt * ((ezy - ez) - (eyn - ey));
        ((real *)a.Bo[1])[g] = Hy[g] - hdt * ((exn - ex) - (ezx - ez));
        ((real *)a.Bo[2])[g] = Hz[g] - hdt * ((eyx - ey) - (exy - ex));
        ex = exn;
        ey = eyn;
    }
}

// ---------------------------------------------------------------------------
// Per-box counts and features
// ---------------------------------------------------------------------------

// Each wave counts a contiguous run of kBoxRun particles.  The particles are
// grouped by tile, so a wave's keys rarely change: a wave-uniform running
// count is kept and flushed with one atomic when the key changes.
constexpr int kBoxRun = 4096;

template <typename real>
__global__ void k_box_counts(Particles<real> P, int np, Geom G, unsigned long long *counts) {
    const int lane = threadIdx.x & 63;
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t p0 = w * kBoxRun;
    if (p0 >= np) return;
    const int p1 = (int)min((int64_t)np, p0 + kBoxRun);
    int run_key = -1;
    unsigned long long run = 0;
    for (int base = (int)p0; base < p1; base += 64) {
        const int p = base + lane;
        int key = -1;
        if (p < p1) {
            int x, y, z;
            unpack_cell(P.cell[p], x, y, z);
            key = box_of_cell(G, x, y, z) * G.nsp + P.sp[p];
        }
        const unsigned long long act = __ballot(key >= 0);
        const int k0 = __shfl(key, 0);
        if (__ballot(key == k0) == act) {
            // the whole wave shares one key
            if (k0 != run_key) {
                if (lane == 0 && run) atomicAdd(&counts[run_key], run);
                run_key = k0;
                run = 0;
            }
            run += (unsigned long long)__popcll(act);
        } else if (key >= 0) {
            wave_count_add(counts, key);
        }
    }
    if (lane == 0 && run) atomicAdd(&counts[run_key], run);
}

// Per-particle pass of the features: per-cell counts, per-box species counts,
// outer-layer counts and the sum of |u|.
template <typename real>
__global__ void k_feat_particles(Particles<real> P, int np, Geom G, const int *box_hi, uint32_t *cellcount,
                                 unsigned long long *spcnt, unsigned long long *edge, double *usum) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    int x, y, z;
    unpack_cell(P.cell[p], x, y, z);
    int b = box_of_cell(G, x, y, z);
    atomicAdd(&cellcount[x + (size_t)G.n[0] * (y + (size_t)G.n[1] * z)], 1u);
    int s = P.sp[p];
    if (s < 2) wave_count_add(spcnt, 2 * b + s);
    const int *lo = G.box_lo + 3 * b, *hi = box_hi + 3 * b;
    bool on = x == lo[0] || x == hi[0] - 1 || y == lo[1] || y == hi[1] - 1 || z == lo[2] || z == hi[2] - 1;
    if (on) wave_count_add(edge, b);
    double ux = P.u[0][p], uy = P.u[1][p], uz = P.u[2][p];
    wave_sum_add(usum, b, sqrt(ux * ux + uy * uy + uz * uz));
}

__global__ void k_feat_boxes(const uint32_t *cellcount, Geom G, const int *box_hi, const unsigned long long *spcnt,
                             const unsigned long long *edge, const double *usum, float *feat) {
    __shared__ unsigned int hist[8];
    __shared__ unsigned int smax;
    int b = blockIdx.x;
    if (threadIdx.x < 8) hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) smax = 0;
    __syncthreads();
    const int *lo = G.box_lo + 3 * b, *hi = box_hi + 3 * b;
    int ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    int ncell = ex * ey * ez;
    unsigned int lh[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned int lmax = 0;
    for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
        int x = lo[0] + q % ex, y = lo[1] + (q / ex) % ey, z = lo[2] + q / (ex * ey);
        unsigned int v = cellcount[x + (size_t)G.n[0] * (y + (size_t)G.n[1] * z)];
        int bin = v == 0 ? 0 : (v == 1 ? 1 : min(7, 31 - __clz(v) + 1));
        // v in [2,3] -> 2, [4,7] -> 3, ... [64, inf) -> 7
        lh[bin] += 1;
        lmax = max(lmax, v);
    }
    for (int i = 0; i < 8; ++i)
        if (lh[i]) atomicAdd(&hist[i], lh[i]);
    atomicMax(&smax, lmax);
    __syncthreads();
    if (threadIdx.x == 0) {
        float *f = feat + 16 * (size_t)b;
        double n0 = (double)spcnt[2 * b], n1 = (double)spcnt[2 * b + 1];
        f[0] = (float)log1p(n0);
        f[1] = (float)log1p(n1);
        for (int i = 0; i < 8; ++i) f[2 + i] = (float)log1p((double)hist[i]);
        f[10] = (float)log((double)ncell);
        f[11] = (float)G.order;
        bool touch = lo[0] == 0 || lo[1] == 0 || lo[2] == 0 || hi[0] == G.n[0] || hi[1] == G.n[1] || hi[2] == G.n[2];
        f[12] = touch ? 1.f : 0.f;
        f[13] = (float)log1p((double)edge[b]);
        f[14] = (float)log1p((double)smax);
        double tot = n0 + n1;
        f[15] = tot > 0 ? (float)(usum[b] / tot) : 0.f;
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------

template <typename real>
static Particles<real> cast(const ParticlesRaw &r) {
    Particles<real> p;
    p.cell = r.cell;
    for (int d = 0; d < 3; ++d) {
        p.f[d] = (real *)r.f[d];
        p.u[d] = (real *)r.u[d];
    }
    p.w = (real *)r.w;
    p.id = r.id;
    p.sp = r.sp;
    return p;
}

static unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_load(int prec, const ParticlesRaw &P, const LoadArgs &a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    if (prec == 8) k_load<double><<<nblk(a.n, 256), 256, 0, st>>>(cast<double>(P), a);
    else k_load<float><<<nblk(a.n, 256), 256, 0, st>>>(cast<float>(P), a);
    return hipGetLastError();
}

hipError_t launch_sort(int prec, const ParticlesRaw &S, const ParticlesRaw &D, int np, const Geom &G,
                       const SortScratch &W, hipStream_t st) {
    int nts = W.nseg;
    size_t ncells = (size_t)nts * G.Tvol;
    k_fill<uint32_t><<<std::min<size_t>(4096, (ncells + 255) / 256), 256, 0, st>>>(W.cellcnt, 0u, ncells);
    if (np > 0) {
        if (prec == 8) k_sort_key<double><<<nblk(np, 256), 256, 0, st>>>(cast<double>(S), np, G, W.cellcnt, W.key, W.rank);
        else k_sort_key<float><<<nblk(np, 256), 256, 0, st>>>(cast<float>(S), np, G, W.cellcnt, W.key, W.rank);
    }
    k_sort_seg<<<nts, G.Tvol, 0, st>>>(W.cellcnt, W.cellstart, W.segtot, G.Tvol);
    if (nts <= 4096) {
        k_scan_single<<<1, 1024, 0, st>>>(W.segtot, W.segstart, nts);
    } else {
        int nblk1 = (nts + 1023) / 1024;  // <= W.scan_cap
        k_scan_bsum<<<nblk1, 1024, 0, st>>>(W.segtot, nts, W.bsum);
        k_scan_single<<<1, 1024, 0, st>>>(W.bsum, W.boff, nblk1);
        k_scan_apply<<<nblk1, 1024, 0, st>>>(W.segtot, nts, W.boff, W.segstart);
    }
    k_sort_levels<<<nts, G.Tvol, 0, st>>>(W.cellcnt, W.cellstart, W.segstart, W.table, G.Tvol);
    if (np > 0) {
        if (prec == 8)
            k_sort_scatter<double><<<nblk(np, 256), 256, 0, st>>>(cast<double>(S), cast<double>(D), np, W.key, W.rank,
                                                                   W.cellstart, W.segstart, W.table, G.Tvol);
        else
            k_sort_scatter<float><<<nblk(np, 256), 256, 0, st>>>(cast<float>(S), cast<float>(D), np, W.key, W.rank,
                                                                 W.cellstart, W.segstart, W.table, G.Tvol);
    }
    return hipGetLastError();
}

hipError_t launch_queue(const int *segstart, int ntiles, int nsp, int chunk, const QueueScratch &Q, hipStream_t st) {
    k_queue_count<<<nblk(ntiles, 256), 256, 0, st>>>(segstart, ntiles, nsp, chunk, Q.ncls, Q.cls_cnt);
    k_queue_scan<<<1, 64, 0, st>>>(Q.cls_cnt, Q.cursor, Q.ncls, Q.queue_bounds);
    k_queue_fill<<<nblk(ntiles, 256), 256, 0, st>>>(segstart, ntiles, nsp, chunk, Q.ncls, Q.cursor, Q.queue);
    return hipGetLastError();
}

hipError_t launch_set_int(int *p, int v, hipStream_t st) {
    k_set_int<<<1, 64, 0, st>>>(p, v);
    return hipGetLastError();
}

hipError_t launch_reset_heads(int *heads, hipStream_t st) {
    k_reset_heads<<<1, 64, 0, st>>>(heads);
    return hipGetLastError();
}

hipError_t launch_fill_f(int prec, void *a, double v, size_t n, hipStream_t st) {
    unsigned g = (unsigned)std::min<size_t>(8192, (n + 255) / 256);
    if (g == 0) return hipSuccess;
    if (prec == 8) k_fill<double><<<g, 256, 0, st>>>((double *)a, v, n);
    else k_fill<float><<<g, 256, 0, st>>>((float *)a, (float)v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *a, size_t n, hipStream_t st) {
    unsigned g = (unsigned)std::min<size_t>(8192, (n + 255) / 256);
    if (g == 0) return hipSuccess;
    k_fill<unsigned long long><<<g, 256, 0, st>>>(a, 0ull, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *a, size_t n, hipStream_t st) {
    unsigned g = (unsigned)std::min<size_t>(8192, (n + 255) / 256);
    if (g == 0) return hipSuccess;
    k_fill<uint32_t><<<g, 256, 0, st>>>(a, 0u, n);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *a, size_t n, hipStream_t st) {
    unsigned g = (unsigned)std::min<size_t>(8192, (n + 255) / 256);
    if (g == 0) return hipSuccess;
    k_fill<double><<<g, 256, 0, st>>>(a, 0.0, n);
    return hipGetLastError();
}

// Table of compiled gather-push-deposit variants.
template <typename real, int M, int TX, int TY, int TZ, int H>
static hipError_t gpd_one(const GpdLaunch &L, hipStream_t st) {
    using C = Cfg<real, M, TX, TY, TZ, H>;
    auto kern = k_gpd<real, M, TX, TY, TZ, H>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(C::lds + 512 * C::qslot));
        if (e != hipSuccess) return e;
        attr = true;
    }
    if (L.block != 256 && L.block != 512) return hipErrorInvalidValue;
    GpdArgs<real> A;
    A.P = cast<real>(L.P);
    A.segstart = L.segstart;
    A.tiles = L.tiles;
    for (int c = 0; c < 6; ++c) A.EB[c] = (const real *)L.EB[c];
    for (int c = 0; c < 3; ++c) A.J[c] = (real *)L.J[c];
    for (int d = 0; d < 3; ++d) A.n[d] = L.n[d];
    A.nsp = L.nsp;
    A.dt = (real)L.dt;
    for (int d = 0; d < 3; ++d) A.bext[d] = (real)L.bext[d];
    for (int s = 0; s < kMaxSpecies; ++s) {
        A.h[s] = (real)L.h[s];
        A.coefq[s] = (real)L.coefq[s];
    }
    A.cycles = L.cycles;
    A.rtc = L.rtc;
    A.slow = L.slow;
    A.mode = L.mode;
    A.tile_base = L.tile_base;
    A.species_only = L.species_only;
    A.queue = L.queue;
    A.queue_bounds = L.queue_bounds;
    A.queue_head = L.queue_head;
    if (L.grid == 0) return hipSuccess;
    kern<<<L.grid, L.block, C::lds + (size_t)L.block * C::qslot, st>>>(A);
    return hipGetLastError();
}

template <typename real, int M>
static hipError_t gpd_tile(const GpdLaunch &L, hipStream_t st) {
    const int *T = L.tile;
    if (L.halo != 1) return hipErrorInvalidValue;
    if (T[0] == 8 && T[1] == 8 && T[2] == 8) return gpd_one<real, M, 8, 8, 8, 1>(L, st);
    if (T[0] == 8 && T[1] == 8 && T[2] == 4) return gpd_one<real, M, 8, 8, 4, 1>(L, st);
    if (T[0] == 8 && T[1] == 4 && T[2] == 4) return gpd_one<real, M, 8, 4, 4, 1>(L, st);
    if (T[0] == 4 && T[1] == 4 && T[2] == 4) return gpd_one<real, M, 4, 4, 4, 1>(L, st);
    return hipErrorInvalidValue;
}

bool gpd_supported(const int tile[3], int halo) {
    if (halo != 1) return false;
    return (tile[0] == 8 && tile[1] == 8 && (tile[2] == 8 || tile[2] == 4)) ||
           (tile[0] == 8 && tile[1] == 4 && tile[2] == 4) || (tile[0] == 4 && tile[1] == 4 && tile[2] == 4);
}

size_t gpd_lds_bytes(int prec, int order, const int tile[3], int halo, int block) {
    int rl_eb = order == 1 ? 1 : 2, rh_eb = order == 3 ? 2 : 1, rl_j = order == 1 ? 1 : 2, rh_j = order == 3 ? 3 : 2;
    size_t neb = 1, nj = 1;
    for (int d = 0; d < 3; ++d) {
        neb *= (size_t)(tile[d] + 2 * halo + rl_eb + rh_eb);
        nj *= (size_t)(tile[d] + 2 * halo + rl_j + rh_j);
    }
    return 6 * neb * (size_t)prec + 3 * nj * sizeof(double) + (size_t)block * (7 * (size_t)prec + sizeof(int));
}

hipError_t launch_gpd(int prec, int order, const GpdLaunch &L, hipStream_t st) {
    if (prec == 8) {
        if (order == 3) return gpd_tile<double, 3>(L, st);
        return order == 2 ? gpd_tile<double, 2>(L, st) : gpd_tile<double, 1>(L, st);
    }
    if (order == 3) return gpd_tile<float, 3>(L, st);
    return order == 2 ? gpd_tile<float, 2>(L, st) : gpd_tile<float, 1>(L, st);
}

// The update writes B^{n+1/2} over the current B buffer, which the
// step no longer needs once the new fields are in the other buffers.
hipError_t launch_yee(int prec, const YeeBuffers &Y, const int n[3], double dt, hipStream_t st) {
    YeeArgs a;
    for (int c = 0; c < 3; ++c) {
        a.E[c] = Y.E[c];
        a.B[c] = Y.B[c];
        a.J[c] = Y.J[c];
        a.Eo[c] = Y.Eo[c];
        a.Bo[c] = Y.Bo[c];
        a.Z[c] = Y.Z[c];
        a.n[c] = n[c];
    }
    a.dt = dt;
    dim3 grd((n[0] + YSX - 1) / YSX, (n[1] + YSY - 1) / YSY, (n[2] + YSZ - 1) / YSZ);
    if (prec == 8) {
        k_yee_bhalf<double><<<grd, 256, 0, st>>>(a);
        k_yee_e<double><<<grd, 256, 0, st>>>(a);
        k_yee_b2<double><<<grd, 256, 0, st>>>(a);
    } else {
        k_yee_bhalf<float><<<grd, 256, 0, st>>>(a);
        k_yee_e<float><<<grd, 256, 0, st>>>(a);
        k_yee_b2<float><<<grd, 256, 0, st>>>(a);
    }
    return hipGetLastError();
}


hipError_t launch_box_counts(int prec, const ParticlesRaw &P, int np, const Geom &G, unsigned long long *counts,
                             hipStream_t st) {
    if (np <= 0) return hipSuccess;
    const int64_t waves = ((int64_t)np + kBoxRun - 1) / kBoxRun;
    const unsigned grid = (unsigned)((waves + 3) / 4);  // four waves per block
    if (prec == 8) k_box_counts<double><<<grid, 256, 0, st>>>(cast<double>(P), np, G, counts);
    else k_box_counts<float><<<grid, 256, 0, st>>>(cast<float>(P), np, G, counts);
    return hipGetLastError();
}

hipError_t launch_features(int prec, const ParticlesRaw &P, int np, const Geom &G, int nb, const int *box_hi,
                           const FeatScratch &S, float *feat, hipStream_t st) {
    if (np > 0) {
        if (prec == 8)
            k_feat_particles<double><<<nblk(np, 256), 256, 0, st>>>(cast<double>(P), np, G, box_hi, S.cellcount, S.spcnt,
                                                                    S.edge, S.usum);
        else
            k_feat_particles<float><<<nblk(np, 256), 256, 0, st>>>(cast<float>(P), np, G, box_hi, S.cellcount, S.spcnt,
                                                                   S.edge, S.usum);
    }
    k_feat_boxes<<<nb, 256, 0, st>>>(S.cellcount, G, box_hi, S.spcnt, S.edge, S.usum, feat);
    return hipGetLastError();
}

}  // namespace pb
