// gfx950 kernels of the PIC step other than the gather-push-deposit: the
// on-device particle loader, the tile sort, the work queue of the persistent
// kernel, the Yee update (Yee 1966: B half step, E full step with -J, B half
// step), and the per-box counts and features used for load balancing.
#include "device_util.hpp"
#include "kernels.hpp"

#include <hip/hip_runtime.h>

namespace pb {

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
// segment either by cell (node_major: the particles of a cell are adjacent,
// so lanes of a wave that share a cell can sum their currents across lanes)
// or by (rank of the particle within its cell, cell) (consecutive particles
// then sit in distinct cells, so the lanes of a wave deposit into distinct
// LDS addresses without summing).  A particle belongs to the box of its cell (that
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
    // Lanes that hold a run of equal keys (a node-major input keeps a
    // node's particles together) take one atomic per run: the run's first
    // lane reserves the run's length and the others count on from it.
    const int lane = (int)__lane_id();
    const unsigned long long active = __ballot(1);  // the inactive lanes are the wave's last
    const uint32_t kprev = (uint32_t)__shfl_up((int)k, 1);
    const unsigned long long starts = __ballot(lane == 0 || kprev != k) | ~active;
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const int first = 63 - __clzll(starts & upto);
    const unsigned long long after = starts & ~upto;
    const int end = after ? __ffsll((long long)after) - 1 : 64;
    uint32_t base = 0;
    if (lane == first) base = atomicAdd(&cellcnt[k], (uint32_t)(end - first));
    base = (uint32_t)__shfl((int)base, first);
    rank[p] = base + (uint32_t)(lane - first);
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

// Moves each particle to its slot (the interleaved order, whose level table
// maps the counting-sort position to the slot).
template <typename real>
__global__ void k_sort_scatter(Particles<real> S, Particles<real> D, int np, const uint32_t *key,
                               const uint32_t *rank, const uint32_t *cellstart, const int *segstart,
                               const uint32_t *table, int Tvol) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    uint32_t k = key[p];
    int ts = (int)(k / (uint32_t)Tvol);
    int idx = segstart[ts] + (int)cellstart[k] + (int)rank[p];
    int d = table ? (int)table[idx] : idx;
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

// Node-major order as a gather: the destination of each particle is written
// to perm (one 4-byte scattered store per particle), then every destination
// slot reads its particle, so that the particle data are written in full
// contiguous lines.
__global__ void k_sort_perm(int np, const uint32_t *key, const uint32_t *rank, const uint32_t *cellstart,
                            const int *segstart, int Tvol, uint32_t *perm) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const uint32_t k = key[p];
    const int ts = (int)(k / (uint32_t)Tvol);
    perm[segstart[ts] + (int)cellstart[k] + (int)rank[p]] = (uint32_t)p;
}

template <typename real>
__global__ void k_sort_gather(Particles<real> S, Particles<real> D, int np, const uint32_t *perm) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= np) return;
    const int p = (int)perm[d];
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

// Reserves cnt consecutive slots of counter arr[key] for every lane with
// want set, with one atomic per distinct key in the wave (adjacent tiles
// mostly share a sub-queue and size class, so per-lane atomics would queue
// on a few addresses).  Every lane of the wave calls it.  Returns the lane's
// first slot (0 for lanes without want).
__device__ inline int wave_reserve(int *arr, int key, int cnt, bool want) {
    const int lane = (int)__lane_id();
    unsigned long long todo = __ballot(want);
    int pos = 0;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int lkey = __shfl(key, leader);
        const bool mine = want && key == lkey;
        const int c = mine ? cnt : 0;
        int incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        const int total = __shfl(incl, 63);
        int base = 0;
        if (lane == leader) base = atomicAdd(&arr[lkey], total);
        base = __shfl(base, leader);
        if (mine) pos = base + incl - c;
        todo &= ~__ballot(mine);
    }
    return pos;
}

__global__ void k_queue_count(const int *segstart, int ntiles, int nsp, int chunk, int ncls, int *cls_cnt) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int n = 0, x = 0;
    if (t < ntiles) {
        n = segstart[(t + 1) * nsp] - segstart[t * nsp];
        if (n > 0) x = sub_queue(segstart, t, ntiles, nsp);
    }
    const int full = n / chunk, rem = n - full * chunk;
    (void)wave_reserve(cls_cnt, x * ncls, full, full > 0);
    (void)wave_reserve(cls_cnt, x * ncls + (rem ? size_class(rem, chunk, ncls) : 0), 1, rem > 0);
}

// Bucket offsets: sub-queue major, size class (largest first) minor.  One
// block with a thread per bucket (kSubQueues * ncls, a multiple of 64 and at
// most 1024); the counts are cleared for the next build.
__global__ void k_queue_scan(int *cls_cnt, int *cursor, int ncls, int *qbounds) {
    __shared__ int sh[17];
    const int i = threadIdx.x;
    const int v = cls_cnt[i];
    int tot;
    const int ex = block_excl_scan(v, sh, tot);
    cursor[i] = ex;
    cls_cnt[i] = 0;
    if (i % ncls == 0) qbounds[i / ncls] = ex;
    if (i == 0) qbounds[kSubQueues] = tot;
}

__global__ void k_queue_fill(const int *segstart, int ntiles, int nsp, int chunk, int ncls, int *cursor,
                             int4 *queue) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int b = 0, n = 0, x = 0;
    if (t < ntiles) {
        b = segstart[t * nsp];
        n = segstart[(t + 1) * nsp] - b;
        if (n > 0) x = sub_queue(segstart, t, ntiles, nsp);
    }
    const int full = n / chunk, rem = n - full * chunk;
    const int pf = wave_reserve(cursor, x * ncls, full, full > 0);
    for (int j = 0; j < full; ++j) queue[pf + j] = make_int4(t, b + j * chunk, b + (j + 1) * chunk, 0);
    const int pr = wave_reserve(cursor, x * ncls + (rem ? size_class(rem, chunk, ncls) : 0), 1, rem > 0);
    if (rem) queue[pr] = make_int4(t, b + full * chunk, b + n, 0);
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
// Yee update in streaming passes.  Each thread updates one cell; its
// neighbours are read through the caches.  X is a half-step B buffer.
//   half:  X = B^{n+1/2} = B^n - dt/2 curl E^n (only when X is not current)
//   E:     E^{n+1} = E^n + dt (curl X - J) into the other E buffer, and the
//          next step's J buffer cleared; z-planes that the deposit left
//          untouched (J occupancy flag 0) are neither read nor cleared
//   B:     B^{n+1} = X - dt/2 curl E^{n+1} into the other B buffer, and
//          X = B^{n+1} - dt/2 curl E^{n+1} = B^{n+3/2}, the next step's half
//          step (the same curl, so the next update skips the half pass)
// Curl of E uses forward differences, curl of B backward ones (Yee cell).
//
// The E and B passes run over lists of z-planes.  The planes are split in
// two parts before each step: those that no deposit of the step can reach
// (no current in the previous step within two planes; particles move less
// than a cell per step, and a particle's stencil at the start of a step was
// covered by the previous step's deposit), updated on a second stream while
// the particle kernel runs, and the rest, updated after it.
// ---------------------------------------------------------------------------

// A Yee work unit is 256 threads over a row segment of 2^lx cells in x and
// 256 / 2^lx rows in y, in one z-plane; the widest segment that divides n_x
// (256, 128 or 64 cells) is used.  Measured on 256^3 cells against 64 x 4
// blocks marching 4 planes: the two passes take 0.264 ms instead of 0.293.
// The half pass launches one block per unit (YSZ planes each); the E and B
// passes run a fixed grid of blocks that step through their plane list's
// units.
constexpr int YSZ = 1;

struct YeeArgs {
    const void *E[3], *B[3], *J[3];
    void *X[3];             // B^{n+1/2} (written by the half pass, read by E; B^{n+3/2} out)
    void *Eo[3], *Bo[3], *Z[3];
    const int *jdirty;      // [nz] 0: plane of J known to be zero
    int *zdirty;            // [nz] the same for Z; reset by the B pass once Z is clear
    const int *planes;      // z-planes of this pass
    const int *nplanes;     // their number (device memory)
    int quiet;              // nonzero: planes no deposit of the step reaches (J, Z not read)
    int n[3];
    int lx;                 // log2 of the block's extent in x
    double dt;
};

// Plane lists of the split update (four lists of nz entries, then four
// counts): 0 and 1 the E and B planes out of the deposit's reach, 2 and 3
// the others.  E of plane k is out of reach when Z (the previous step's
// current) is clear on planes k-2..k+2.  B of plane k reads E^{n+1} of
// planes k and k+1, and its new half-step B is read by the E update of plane
// k+1: it joins the early part only when E of both planes does.  split = 0
// puts every plane in lists 2 and 3.  One block of 1024 threads; it also
// rewinds the persistent work queue's sub-queue heads (heads non-null), as
// it runs ahead of the particle kernel.
__global__ __launch_bounds__(1024) void k_yee_class(const int *zdirty, int nz, int split, int *lists, int *heads) {
    __shared__ int wsum[16][4];
    __shared__ int base[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int *cnt = lists + 4 * (size_t)nz;
    if (heads && tid < kSubQueues) heads[tid] = 0;
    if (tid < 4) base[tid] = 0;
    __syncthreads();
    for (int k0 = 0; k0 < nz; k0 += 1024) {
        const int k = k0 + tid;
        bool qe = false, qb = false;
        if (k < nz && split) {
            bool quiet[2] = {true, true};
            for (int d = -2; d <= 3; ++d) {
                const int q = ((k + d) % nz + nz) % nz;
                const bool z = zdirty[q] == 0;
                if (d <= 2) quiet[0] = quiet[0] && z;
                if (d >= -1) quiet[1] = quiet[1] && z;
            }
            qe = quiet[0];
            qb = quiet[0] && quiet[1];
        }
        const bool in[4] = {k < nz && qe, k < nz && qb, k < nz && !qe, k < nz && !qb};
        unsigned long long m[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) m[l] = __ballot(in[l]);
        if (lane == 0)
#pragma unroll
            for (int l = 0; l < 4; ++l) wsum[w][l] = __popcll(m[l]);
        __syncthreads();
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            if (!in[l]) continue;
            int off = base[l] + __popcll(m[l] & ((1ull << lane) - 1ull));
            for (int v = 0; v < w; ++v) off += wsum[v][l];
            lists[(size_t)l * nz + off] = k;
        }
        __syncthreads();
        if (tid < 4) {
            int t = 0;
            for (int v = 0; v < 16; ++v) t += wsum[v][tid];
            base[tid] += t;
        }
        __syncthreads();
    }
    if (tid < 4) cnt[tid] = base[tid];
}

// Work units of a pass over a plane list: unit u is row segment u mod P of
// plane list[u / P] (P segments per plane).  The block steps through units
// u = blockIdx.x + i gridDim.x; the next unit's plane is loaded before the
// current unit is computed.
struct YeeUnits {
    int P, gx, nunit, stride;
    int u, k;  // current unit and its plane
    __device__ __forceinline__ YeeUnits(const YeeArgs &a) {
        gx = (a.n[0] + (1 << a.lx) - 1) >> a.lx;
        P = gx * ((a.n[1] + (256 >> a.lx) - 1) / (256 >> a.lx));
        nunit = P * *a.nplanes;
        stride = gridDim.x;
        u = blockIdx.x;
        k = u < nunit ? a.planes[u / P] : 0;
    }
    // the cell of this thread in unit u
    __device__ __forceinline__ void cell(const YeeArgs &a, int &x, int &y) const {
        const int r = u % P, by = r / gx, bx = r - by * gx;
        x = (bx << a.lx) + (int)(threadIdx.x & ((1u << a.lx) - 1u));
        y = by * (256 >> a.lx) + (int)(threadIdx.x >> a.lx);
    }
};

template <typename real>
__global__ __launch_bounds__(256) void k_yee_bhalf(YeeArgs a) {
    const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
    const int x = ((int)blockIdx.x << a.lx) + (int)(threadIdx.x & ((1u << a.lx) - 1u));
    const int y = (int)blockIdx.y * (256 >> a.lx) + (int)(threadIdx.x >> a.lx);
    if (x >= nx || y >= ny) return;
    const int z0 = blockIdx.z * YSZ, z1 = min(nz, z0 + YSZ);
    const real hdt = (real)(0.5 * a.dt);
    const real *Ex = (const real *)a.E[0], *Ey = (const real *)a.E[1], *Ez = (const real *)a.E[2];
    const real *Bx = (const real *)a.B[0], *By = (const real *)a.B[1], *Bz = (const real *)a.B[2];
    real *Xx = (real *)a.X[0], *Xy = (real *)a.X[1], *Xz = (real *)a.X[2];
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
        Xx[g] = Bx[g] - hdt * cx;
        Xy[g] = By[g] - hdt * cy;
        Xz[g] = Bz[g] - hdt * cz;
        ex = exn;
        ey = eyn;
    }
}

template <typename real>
__global__ __launch_bounds__(256) void k_yee_e(YeeArgs a) {
    const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
    const real dt = (real)a.dt;
    const real *Ex = (const real *)a.E[0], *Ey = (const real *)a.E[1], *Ez = (const real *)a.E[2];
    const real *Jx = (const real *)a.J[0], *Jy = (const real *)a.J[1], *Jz = (const real *)a.J[2];
    const real *Hx = (const real *)a.X[0], *Hy = (const real *)a.X[1], *Hz = (const real *)a.X[2];
    const size_t sxy = (size_t)nx * ny;
    for (YeeUnits w(a); w.u < w.nunit;) {
        const int k = w.k;
        int x, y;
        w.cell(a, x, y);
        const int un = w.u + w.stride;
        w.k = un < w.nunit ? a.planes[un / w.P] : 0;
        w.u = un;
        if (x >= nx || y >= ny) continue;
        const int xm = x == 0 ? nx - 1 : x - 1, ym = y == 0 ? ny - 1 : y - 1;
        const size_t c0 = (size_t)x + (size_t)nx * y, cxm = (size_t)xm + (size_t)nx * y, cym = (size_t)x + (size_t)nx * ym;
        const size_t gk = sxy * k, g = c0 + gk, gm = sxy * (k == 0 ? nz - 1 : k - 1);
        const bool jd = !a.quiet && a.jdirty[k] != 0, zd = !a.quiet && a.zdirty[k] != 0;
        const real hx_m = Hx[c0 + gm], hy_m = Hy[c0 + gm];
        const real hx = Hx[g], hy = Hy[g], hz = Hz[g];
        const real hzym = Hz[cym + gk], hzxm = Hz[cxm + gk], hyxm = Hy[cxm + gk], hxym = Hx[cym + gk];
        real jx = (real)0, jy = (real)0, jz = (real)0;
        if (jd) {
            jx = Jx[g];
            jy = Jy[g];
            jz = Jz[g];
        }
        // every load before the first store (the output buffers could alias
        // the inputs as far as the compiler knows); the stores carry the
        // non-temporal hint, which leaves the caches to the planes still
        // being read (and to the particle kernel beside the early part)
        const real ex = Ex[g], ey = Ey[g], ez = Ez[g];
        __builtin_nontemporal_store(ex + dt * (((hz - hzym) - (hy - hy_m)) - jx), &((real *)a.Eo[0])[g]);
        __builtin_nontemporal_store(ey + dt * (((hx - hx_m) - (hz - hzxm)) - jy), &((real *)a.Eo[1])[g]);
        __builtin_nontemporal_store(ez + dt * (((hy - hyxm) - (hx - hxym)) - jz), &((real *)a.Eo[2])[g]);
        if (zd) {
            __builtin_nontemporal_store((real)0, &((real *)a.Z[0])[g]);
            __builtin_nontemporal_store((real)0, &((real *)a.Z[1])[g]);
            __builtin_nontemporal_store((real)0, &((real *)a.Z[2])[g]);
        }
    }
}

template <typename real>
__global__ __launch_bounds__(256) void k_yee_b2(YeeArgs a) {
    const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
    const real hdt = (real)(0.5 * a.dt);
    const real *Ex = (const real *)a.Eo[0], *Ey = (const real *)a.Eo[1], *Ez = (const real *)a.Eo[2];
    real *Hx = (real *)a.X[0], *Hy = (real *)a.X[1], *Hz = (real *)a.X[2];
    const size_t sxy = (size_t)nx * ny;
    for (YeeUnits w(a); w.u < w.nunit;) {
        const int k = w.k;
        int x, y;
        w.cell(a, x, y);
        const int un = w.u + w.stride;
        w.k = un < w.nunit ? a.planes[un / w.P] : 0;
        w.u = un;
        if (x >= nx || y >= ny) continue;
        const int xp = x + 1 == nx ? 0 : x + 1, yp = y + 1 == ny ? 0 : y + 1;
        const size_t col = (size_t)x + (size_t)nx * y, colx = (size_t)xp + (size_t)nx * y,
                     coly = (size_t)x + (size_t)nx * yp;
        const size_t gk = sxy * k, gn = sxy * (k + 1 == nz ? 0 : k + 1), g = col + gk;
        const real ex = Ex[g], ey = Ey[g];
        const real exn = Ex[col + gn], eyn = Ey[col + gn];
        const real ez = Ez[g];
        const real eyx = Ey[colx + gk], ezx = Ez[colx + gk];
        const real exy = Ex[coly + gk], ezy = Ez[coly + gk];
        const real cx = (ezy - ez) - (eyn - ey);
        const real cy = (exn - ex) - (ezx - ez);
        const real cz = (eyx - ey) - (exy - ex);
        const real bx = Hx[g] - hdt * cx, by = Hy[g] - hdt * cy, bz = Hz[g] - hdt * cz;
        // non-temporal stores, as in the E pass
        __builtin_nontemporal_store(bx, &((real *)a.Bo[0])[g]);
        __builtin_nontemporal_store(by, &((real *)a.Bo[1])[g]);
        __builtin_nontemporal_store(bz, &((real *)a.Bo[2])[g]);
        __builtin_nontemporal_store(bx - hdt * cx, &Hx[g]);
        __builtin_nontemporal_store(by - hdt * cy, &Hy[g]);
        __builtin_nontemporal_store(bz - hdt * cz, &Hz[g]);
    }
    // the E pass (earlier on the stream) has cleared Z: its planes are zero
    // (the early part's planes were clear already); done after the loop, so
    // that the loop's plane-list loads stay scalar loads
    if (!a.quiet)
        for (int zi = (int)(blockIdx.x * blockDim.x + threadIdx.x); zi < *a.nplanes;
             zi += (int)(gridDim.x * blockDim.x))
            a.zdirty[a.planes[zi]] = 0;
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
// outer-layer counts and the sum of |u|.  As in k_box_counts, each wave walks
// a run of kBoxRun particles and keeps wave-uniform running sums while all
// its lanes see one box (the particles are grouped by tile), so that the
// per-box atomics, which every wave of a box would otherwise take on the same
// addresses, are taken about once per run.  The per-cell counts of the
// block's particles are gathered in an LDS hash table (open addressing,
// kFeatSlots slots, at most kFeatProbes probes, else a global atomic) and
// added to the global counts once per distinct cell.
constexpr int kFeatSlots = 2048;
constexpr int kFeatProbes = 16;
constexpr uint32_t kFeatEmpty = 0xFFFFFFFFu;
static_assert(kFeatSlots == 1 << 11, "the slot hash takes the top 11 bits");

template <typename real>
__global__ __launch_bounds__(256) void k_feat_particles(Particles<real> P, int np, Geom G, const int *box_hi,
                                                        uint32_t *cellcount, unsigned long long *spcnt,
                                                        unsigned long long *edge, double *usum) {
    __shared__ uint32_t sKey[kFeatSlots], sCnt[kFeatSlots];
    for (int i = threadIdx.x; i < kFeatSlots; i += blockDim.x) {
        sKey[i] = kFeatEmpty;
        sCnt[i] = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t p0 = w * kBoxRun;
    const int p1 = (int)min((int64_t)np, p0 + kBoxRun);
    int rb = -1;  // box of the running sums
    unsigned long long r0 = 0, r1 = 0, re = 0;
    double ru = 0.0;
    auto flush = [&]() {
        if (lane == 0 && rb >= 0) {
            if (r0) atomicAdd(&spcnt[2 * rb], r0);
            if (r1) atomicAdd(&spcnt[2 * rb + 1], r1);
            if (re) atomicAdd(&edge[rb], re);
            if (ru != 0.0) unsafeAtomicAdd(&usum[rb], ru);
        }
    };
    for (int base = (int)p0; base < p1; base += 64) {
        const int p = base + lane;
        int b = -1, s = 0;
        bool on = false;
        double um = 0.0;
        if (p < p1) {
            int x, y, z;
            unpack_cell(P.cell[p], x, y, z);
            b = box_of_cell(G, x, y, z);
            const uint32_t key = (uint32_t)x + (uint32_t)G.n[0] * ((uint32_t)y + (uint32_t)G.n[1] * (uint32_t)z);
            uint32_t h = (key * 2654435761u) >> (32 - 11);
            bool done = key == kFeatEmpty;  // the last cell of a domain of 2^32 cells goes to the global array
            if (done) atomicAdd(&cellcount[key], 1u);
            for (int q = 0; q < kFeatProbes && !done; ++q, h = (h + 1) & (kFeatSlots - 1)) {
                uint32_t k = sKey[h];
                if (k == kFeatEmpty) k = atomicCAS(&sKey[h], kFeatEmpty, key);
                if (k == kFeatEmpty || k == key) {
                    atomicAdd(&sCnt[h], 1u);
                    done = true;
                }
            }
            if (!done) atomicAdd(&cellcount[key], 1u);  // table full along the probe sequence
            s = P.sp[p];
            const int *lo = G.box_lo + 3 * b, *hi = box_hi + 3 * b;
            on = x == lo[0] || x == hi[0] - 1 || y == lo[1] || y == hi[1] - 1 || z == lo[2] || z == hi[2] - 1;
            const double ux = P.u[0][p], uy = P.u[1][p], uz = P.u[2][p];
            um = sqrt(ux * ux + uy * uy + uz * uz);
        }
        const unsigned long long act = __ballot(b >= 0);
        const int b0 = __shfl(b, 0);
        if (__ballot(b == b0) == act) {
            // the whole wave is in one box
            if (b0 != rb) {
                flush();
                rb = b0;
                r0 = r1 = re = 0;
                ru = 0.0;
            }
            r0 += (unsigned long long)__popcll(__ballot(b >= 0 && s == 0));
            r1 += (unsigned long long)__popcll(__ballot(b >= 0 && s == 1));
            re += (unsigned long long)__popcll(__ballot(on));
            double t = um;
            for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
            ru += t;
        } else if (b >= 0) {
            if (s < 2) wave_count_add(spcnt, 2 * b + s);
            if (on) wave_count_add(edge, b);
            wave_sum_add(usum, b, um);
        }
    }
    flush();
    __syncthreads();
    for (int i = threadIdx.x; i < kFeatSlots; i += blockDim.x)
        if (sCnt[i]) atomicAdd(&cellcount[sKey[i]], sCnt[i]);
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
                       const SortScratch &W, bool node_major, hipStream_t st) {
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
    const uint32_t *table = nullptr;
    if (!node_major) {
        k_sort_levels<<<nts, G.Tvol, 0, st>>>(W.cellcnt, W.cellstart, W.segstart, W.table, G.Tvol);
        table = W.table;
    }
    if (np > 0 && node_major) {
        // W.table (capacity entries) serves as the permutation
        k_sort_perm<<<nblk(np, 256), 256, 0, st>>>(np, W.key, W.rank, W.cellstart, W.segstart, G.Tvol, W.table);
        if (prec == 8) k_sort_gather<double><<<nblk(np, 256), 256, 0, st>>>(cast<double>(S), cast<double>(D), np, W.table);
        else k_sort_gather<float><<<nblk(np, 256), 256, 0, st>>>(cast<float>(S), cast<float>(D), np, W.table);
    } else if (np > 0) {
        if (prec == 8)
            k_sort_scatter<double><<<nblk(np, 256), 256, 0, st>>>(cast<double>(S), cast<double>(D), np, W.key, W.rank,
                                                                   W.cellstart, W.segstart, table, G.Tvol);
        else
            k_sort_scatter<float><<<nblk(np, 256), 256, 0, st>>>(cast<float>(S), cast<float>(D), np, W.key, W.rank,
                                                                 W.cellstart, W.segstart, table, G.Tvol);
    }
    return hipGetLastError();
}

hipError_t launch_queue(const int *segstart, int ntiles, int nsp, int chunk, const QueueScratch &Q, hipStream_t st) {
    if (Q.ncls < 8 || Q.ncls > 1024 / kSubQueues || (kSubQueues * Q.ncls) % 64) return hipErrorInvalidValue;
    k_queue_count<<<nblk(ntiles, 256), 256, 0, st>>>(segstart, ntiles, nsp, chunk, Q.ncls, Q.cls_cnt);
    k_queue_scan<<<1, kSubQueues * Q.ncls, 0, st>>>(Q.cls_cnt, Q.cursor, Q.ncls, Q.queue_bounds);
    k_queue_fill<<<nblk(ntiles, 256), 256, 0, st>>>(segstart, ntiles, nsp, chunk, Q.ncls, Q.cursor, Q.queue);
    return hipGetLastError();
}

hipError_t launch_set_int(int *p, int v, hipStream_t st) {
    k_set_int<<<1, 64, 0, st>>>(p, v);
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

hipError_t launch_fill_u32(uint32_t *a, size_t n, hipStream_t st, uint32_t v) {
    unsigned g = (unsigned)std::min<size_t>(8192, (n + 255) / 256);
    if (g == 0) return hipSuccess;
    k_fill<uint32_t><<<g, 256, 0, st>>>(a, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *a, size_t n, hipStream_t st) {
    unsigned g = (unsigned)std::min<size_t>(8192, (n + 255) / 256);
    if (g == 0) return hipSuccess;
    k_fill<double><<<g, 256, 0, st>>>(a, 0.0, n);
    return hipGetLastError();
}


static int yee_lx(const int n[3]) { return n[0] % 256 == 0 ? 8 : (n[0] % 128 == 0 ? 7 : 6); }

static YeeArgs yee_args(const YeeBuffers &Y, const int n[3], double dt) {
    YeeArgs a;
    for (int c = 0; c < 3; ++c) {
        a.E[c] = Y.E[c];
        a.B[c] = Y.B[c];
        a.J[c] = Y.J[c];
        a.X[c] = Y.X[c];
        a.Eo[c] = Y.Eo[c];
        a.Bo[c] = Y.Bo[c];
        a.Z[c] = Y.Z[c];
        a.n[c] = n[c];
    }
    a.jdirty = Y.jdirty;
    a.zdirty = Y.zdirty;
    a.planes = nullptr;
    a.nplanes = nullptr;
    a.quiet = 0;
    a.lx = yee_lx(n);
    a.dt = dt;
    return a;
}

static dim3 yee_grid(const int n[3]) {
    const int lx = yee_lx(n), sx = 1 << lx, sy = 256 >> lx;
    return dim3((n[0] + sx - 1) / sx, (n[1] + sy - 1) / sy, (n[2] + YSZ - 1) / YSZ);
}

hipError_t launch_yee_half(int prec, const YeeBuffers &Y, const int n[3], double dt, hipStream_t st) {
    YeeArgs a = yee_args(Y, n, dt);
    if (prec == 8) k_yee_bhalf<double><<<yee_grid(n), 256, 0, st>>>(a);
    else k_yee_bhalf<float><<<yee_grid(n), 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_yee_class(const YeeBuffers &Y, int nz, bool split, int *heads, hipStream_t st) {
    k_yee_class<<<1, 1024, 0, st>>>(Y.zdirty, nz, split ? 1 : 0, Y.lists, heads);
    return hipGetLastError();
}

hipError_t launch_yee(int prec, const YeeBuffers &Y, const int n[3], double dt, int part, unsigned grid,
                      hipStream_t st) {
    if (grid == 0) return hipSuccess;
    YeeArgs a = yee_args(Y, n, dt);
    a.quiet = part == 0 ? 1 : 0;
    const int le = part == 0 ? 0 : 2;  // the part's E list; its B list follows
    const size_t nz = (size_t)n[2];
    YeeArgs b = a;
    a.planes = Y.lists + le * nz;
    a.nplanes = Y.lists + 4 * nz + le;
    b.planes = Y.lists + (le + 1) * nz;
    b.nplanes = Y.lists + 4 * nz + le + 1;
    if (prec == 8) {
        k_yee_e<double><<<grid, 256, 0, st>>>(a);
        k_yee_b2<double><<<grid, 256, 0, st>>>(b);
    } else {
        k_yee_e<float><<<grid, 256, 0, st>>>(a);
        k_yee_b2<float><<<grid, 256, 0, st>>>(b);
    }
    return hipGetLastError();
}

// Particles of species s whose ids are in the ascending list q[0, n): each
// found particle's cell, offsets and momentum go to slot k of the outputs,
// k its id's position in q, and found[k] is set.
template <typename real>
__global__ void k_find_ids(Particles<real> P, int np, int s, const int64_t *q, int n, uint32_t *cell, real *f,
                           real *u, int *found) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np || P.sp[p] != s) return;
    const int64_t id = P.id[p];
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (q[mid] < id) lo = mid + 1;
        else hi = mid;
    }
    if (lo >= n || q[lo] != id) return;
    cell[lo] = P.cell[p];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        f[3 * lo + d] = P.f[d][p];
        u[3 * lo + d] = P.u[d][p];
    }
    found[lo] = 1;
}

hipError_t launch_find_ids(int prec, const ParticlesRaw &P, int np, int s, const int64_t *q, int n, uint32_t *cell,
                           void *f, void *u, int *found, hipStream_t st) {
    if (np <= 0 || n <= 0) return hipSuccess;
    if (prec == 8)
        k_find_ids<double><<<nblk(np, 256), 256, 0, st>>>(cast<double>(P), np, s, q, n, cell, (double *)f,
                                                           (double *)u, found);
    else
        k_find_ids<float><<<nblk(np, 256), 256, 0, st>>>(cast<float>(P), np, s, q, n, cell, (float *)f, (float *)u,
                                                         found);
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
        const int64_t waves = ((int64_t)np + kBoxRun - 1) / kBoxRun;
        const unsigned grid = (unsigned)((waves + 3) / 4);  // four waves per block
        if (prec == 8)
            k_feat_particles<double><<<grid, 256, 0, st>>>(cast<double>(P), np, G, box_hi, S.cellcount, S.spcnt,
                                                           S.edge, S.usum);
        else
            k_feat_particles<float><<<grid, 256, 0, st>>>(cast<float>(P), np, G, box_hi, S.cellcount, S.spcnt, S.edge,
                                                          S.usum);
    }
    k_feat_boxes<<<nb, 256, 0, st>>>(S.cellcount, G, box_hi, S.spcnt, S.edge, S.usum, feat);
    return hipGetLastError();
}

}  // namespace pb
