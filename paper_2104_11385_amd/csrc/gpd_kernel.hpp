// gfx950 gather-push-deposit kernel of the PIC step, with the in-kernel
// per-box clock costs, and its launcher (templates; gpd_inst.hip
// instantiates them per precision and shape order).
//
// Numerical methods (the paper names the PIC scheme only in words, Sec. 2.1):
//   shapes   centred B-splines of order 1, 2 or 3;
//   gather   each component interpolated at its own Yee stagger with the same
//            order-m spline;
//   push     relativistic Boris rotation (Boris 1970; Birdsall & Langdon);
//   deposit  Esirkepov (2001) charge-conserving density decomposition.
// Per-box costs follow Sec. 2.2 and Fig. 2a: a device clock is read around
// the compute-intensive work, summed on chip, then added once per block to a
// global per-box counter.
//
// Structure: a block takes a work item (a tile's particles, all species),
// stages the tile's E/B window in LDS and accumulates J in an FP64 LDS
// window that it adds to the global J at the end of the item.  Each wave
// walks its own 64-particle runs of the item.  With R (node-major particle
// order), the currents of lanes whose particles keep a common reference node
// are summed across the lanes of each 16-lane row (and across one row
// boundary) before one LDS add per run; particles that change node wait in a
// per-wave queue for a wider deposit on full waves.  A particle whose
// stencils leave the windows (it drifted beyond the halo since the last
// sort) is listed, and a second kernel pushes the listed particles through
// the global arrays after the tile kernel.
#pragma once

#include "device_util.hpp"
#include "kernels.hpp"

#include <hip/hip_runtime.h>

#include <climits>
#include <type_traits>

namespace pb {

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
// CM selects the components (bit 0: Jx, 1: Jy, 2: Jz).
template <typename real, int M, int L, int CM = 7, typename Acc>
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
    for (int c = 0; c < ((CM & 1) ? L : 0); ++c)
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
    for (int c = 0; c < ((CM & 2) ? L : 0); ++c)
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
    for (int b = 0; b < ((CM & 4) ? L : 0); ++b)
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
        // opaque to the optimiser: otherwise it rebases the six components'
        // taps on one register, and the negative offsets that leaves need an
        // add each (LDS reads take only non-negative immediate offsets)
        asm("" : "+v"(base));
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
        asm("" : "+v"(base));  // as in LdsEB::begin
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
    int *jdirty;
    int n[3], r[3];
    int ix[5], iy[5], iz[5];
    __device__ __forceinline__ void begin(int sx, int sy, int sz) {
        for (int q = 0; q < 5; ++q) {
            ix[q] = wrap_any(r[0] + sx + q, n[0]);
            iy[q] = wrap_any(r[1] + sy + q, n[1]);
            iz[q] = wrap_any(r[2] + sz + q, n[2]);
            jdirty[iz[q]] = 1;
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
    // The particle arrays are streamed once per step: their loads and stores
    // carry the non-temporal hint, which leaves the caches to the field
    // windows and the current.
    __device__ __forceinline__ void load(const Particles<real> &P, int p) {
        cell = __builtin_nontemporal_load(&P.cell[p]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            f[d] = __builtin_nontemporal_load(&P.f[d][p]);
            u[d] = __builtin_nontemporal_load(&P.u[d][p]);
        }
        w = __builtin_nontemporal_load(&P.w[p]);
    }
    // Writes the moved particle (cell, offsets, momentum) back to slot p.
    __device__ __forceinline__ void store(const Particles<real> &P, int p) const {
        __builtin_nontemporal_store(cell, &P.cell[p]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            __builtin_nontemporal_store(f[d], &P.f[d][p]);
            __builtin_nontemporal_store(u[d], &P.u[d][p]);
        }
    }
    // A stand-in for a lane past the item's end: a particle of zero weight
    // at rest at the tile origin, whose current and queue entries vanish.
    __device__ __forceinline__ void blank(uint32_t origin) {
        cell = origin;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            f[d] = (real)0.25;
            u[d] = (real)0;
        }
        w = (real)0;
    }
    // Makes the registers count as used here, so the compiler waits for the
    // loads at this point.  Used on the first particle before the loop
    // (otherwise that path's pending loads merge into the loop's and every
    // iteration stalls on the next particle's first load) and on the next
    // particle before the current one's stores.
    __device__ __forceinline__ void settle() const {
        asm volatile("" : : "v"(cell));
#pragma unroll
        for (int d = 0; d < 3; ++d) asm volatile("" : : "v"(f[d]), "v"(u[d]));
        asm volatile("" : : "v"(w));
    }
};

// A particle that changed its reference node inside the staged window: its
// wider deposit waits in the wave's queue so that it runs with the other
// queued particles on full waves rather than on otherwise idle lanes.
// The same record carries a particle that kept its node when its current
// is summed with its lane neighbours' (keep).
template <typename real>
struct Deferred {
    bool want, keep;
    int rel;          // packed window-relative reference node, +8 per byte
    real d0[3], D[3], coef;
};

// Reference point of a particle at cell c, offset f: the cell (orders 1
// and 3) or the nearest node (order 2), and the offset d0 from it.
template <typename real, int M>
__device__ __forceinline__ void reference(const int c[3], const real f[3], int ref[3], real d0[3]) {
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
}

// Relativistic Boris rotation of u in the gathered fields EB (B without its
// uniform external part, added here), and the displacement D over dt.
template <typename real>
__device__ __forceinline__ void boris_move(const GpdArgs<real> &A, real hq, real EB[6], real u[3], real D[3]) {
    // the arrays hold B minus its uniform external part (whose curl is zero)
    EB[3] += A.bext[0];
    EB[4] += A.bext[1];
    EB[5] += A.bext[2];
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
    D[0] = A.dt * u[0] * gi;
    D[1] = A.dt * u[1] * gi;
    D[2] = A.dt * u[2] * gi;
}

// New canonical position after the displacement D: cell + offset in [0, 1),
// periodic wrap (a step below zero so small that x + 1 rounds to 1 keeps the
// cell, at offset 0); selects rather than branches.
template <typename real>
__device__ __forceinline__ void advance(const GpdArgs<real> &A, int c[3], const real f[3], const real D[3],
                                        const real u[3], PState<real> &out) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const real x = f[d] + D[d];
        // |D| < 1: the floor is -1, 0 or 1, and x - floor(x) rounds as
        // x + 1 or x - 1 would
        const real fl = floor(x);
        real y = x - fl;
        int k = (int)fl;
        const bool stay = y >= (real)1;
        y = stay ? (real)0 : y;
        k = stay ? 0 : k;
        int cc = c[d] + k;
        cc = cc < 0 ? cc + A.n[d] : (cc >= A.n[d] ? cc - A.n[d] : cc);
        c[d] = cc;
        out.f[d] = y;
        out.u[d] = u[d];
    }
    out.cell = pack_cell(c[0], c[1], c[2]);
}

// Push of one particle whose gather and deposit stencils lie in the tile's
// staged LDS windows; returns false when they do not.  Such a particle is
// computed on a harmless in-window reference, its deposit record is left
// empty (df as given), and the caller drops its results and leaves it to
// the global-path kernel.
template <typename real, int M, int TX, int TY, int TZ, int H, bool R>
__device__ __forceinline__ bool push_staged(const GpdArgs<real> &A, const PState<real> &ps, const TileDesc &td,
                                            real hq, real cq, const real *sEB, double *sJ, Deferred<real> &df,
                                            PState<real> &out) {
    using C = Cfg<real, M, TX, TY, TZ, H>;
    int c[3];
    unpack_cell(ps.cell, c[0], c[1], c[2]);
    const real f[3] = {ps.f[0], ps.f[1], ps.f[2]};
    real u[3] = {ps.u[0], ps.u[1], ps.u[2]};
    int ref[3];
    real d0[3];
    reference<real, M>(c, f, ref, d0);
    const int T[3] = {TX, TY, TZ};
    const int org[3] = {td.x0, td.y0, td.z0};
    int rel[3];
    bool fast = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        rel[d] = wrap_rel(ref[d] - org[d], H, A.n[d]);
        fast = fast && rel[d] <= T[d] + H - 1;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) rel[d] = fast ? rel[d] : 0;

    GatherW<real, M> GW[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) GW[d].set(d0[d]);
    real EB[6];
    LdsEB<real, C> acc{sEB, (rel[0] + H + C::RL_EB) + C::EX * ((rel[1] + H + C::RL_EB) + C::EY * (rel[2] + H + C::RL_EB)), 0};
    gather6<real, M>(acc, GW, EB);
    real D[3];
    boris_move(A, hq, EB, u, D);

    // Esirkepov deposit
    const real coef = cq * ps.w;
    const bool moved = leaves_ref<real, M>(d0[0], D[0]) || leaves_ref<real, M>(d0[1], D[1]) ||
                       leaves_ref<real, M>(d0[2], D[2]);
    // every lane's record is complete (finite values), whatever path it takes
    df.rel = (rel[0] + 8) | ((rel[1] + 8) << 8) | ((rel[2] + 8) << 16);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        df.d0[d] = d0[d];
        df.D[d] = D[d];
    }
    df.coef = coef;
    if (fast) {
        if (moved || R) {
            df.want = moved;
            df.keep = !moved;
        } else {
            DepW<real, M> DW[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) DW[d].set_kept(d0[d], D[d]);
            LdsJ<real, C> jacc{sJ, (rel[0] + H + C::RL_J) + C::JX * ((rel[1] + H + C::RL_J) + C::JY * (rel[2] + H + C::RL_J)), 0};
            deposit3<real, M, M + 1>(jacc, DW, coef);
        }
    }
    advance(A, c, f, D, u, out);
    return fast;
}

// Push of one particle through the global arrays (gather with periodic wrap,
// deposit by global atomics): particles beyond their tile's staged windows,
// and every particle when staging is off.
template <typename real, int M>
__device__ __forceinline__ void push_global(const GpdArgs<real> &A, const PState<real> &ps, real hq, real cq,
                                            PState<real> &out) {
    int c[3];
    unpack_cell(ps.cell, c[0], c[1], c[2]);
    const real f[3] = {ps.f[0], ps.f[1], ps.f[2]};
    real u[3] = {ps.u[0], ps.u[1], ps.u[2]};
    int ref[3];
    real d0[3];
    reference<real, M>(c, f, ref, d0);
    GatherW<real, M> GW[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) GW[d].set(d0[d]);
    real EB[6];
    {
        GlobEB<real> acc;
        acc.EB = A.EB;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            acc.n[d] = A.n[d];
            acc.r[d] = ref[d];
        }
        gather6<real, M>(acc, GW, EB);
    }
    real D[3];
    boris_move(A, hq, EB, u, D);
    {
        DepW<real, M> DW[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) DW[d].set(d0[d], D[d]);
        GlobJ<real> acc;
        acc.J = A.J;
        acc.jdirty = A.jdirty;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            acc.n[d] = A.n[d];
            acc.r[d] = ref[d];
        }
        deposit3<real, M, M + 2>(acc, DW, cq * ps.w);
    }
    advance(A, c, f, D, u, out);
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

// Register image of one particle's kept-node current (window of M + 1 nodes
// per dimension); entry (comp, a, b, c) is used when the index along comp's
// own axis is below M.
template <typename real, int L>
struct RegJ {
    real v[3][L][L][L];
    __device__ __forceinline__ void begin(int, int, int) {}
    __device__ __forceinline__ void add(int comp, int a, int b, int c, real x) { v[comp][a][b][c] = x; }
    static constexpr bool used(int comp, int a, int b, int c) {
        return (comp == 0 ? a : (comp == 1 ? b : c)) < L - 1;
    }
};

// One component of the run sums; lanes with lead set add where they end a
// run (their run lies in the staged window).
template <typename real, int M, int COMP, typename Acc>
__device__ __forceinline__ void runs_comp(Acc &J, const DepW<real, M> DW[3], real coef, const RowRuns<real> &rr,
                                          bool lead) {
    constexpr int L = M + 1;
    RegJ<real, L> acc;
    deposit3<real, M, L, 1 << COMP>(acc, DW, coef);
    if constexpr (std::is_same<real, float>::value) {
        // the M L^2 used entries, packed
        float f[M * L * L];
        int k = 0;
#pragma unroll
        for (int c = 0; c < L; ++c)
#pragma unroll
            for (int b = 0; b < L; ++b)
#pragma unroll
                for (int a = 0; a < L; ++a)
                    if (RegJ<real, L>::used(COMP, a, b, c)) f[k++] = acc.v[COMP][a][b][c];
        rr.sum_n(f);
        k = 0;
#pragma unroll
        for (int c = 0; c < L; ++c)
#pragma unroll
            for (int b = 0; b < L; ++b)
#pragma unroll
                for (int a = 0; a < L; ++a)
                    if (RegJ<real, L>::used(COMP, a, b, c)) acc.v[COMP][a][b][c] = f[k++];
    } else {
#pragma unroll
        for (int c = 0; c < L; ++c)
#pragma unroll
            for (int b = 0; b < L; ++b)
#pragma unroll
                for (int a = 0; a < L; ++a)
                    if (RegJ<real, L>::used(COMP, a, b, c)) acc.v[COMP][a][b][c] = rr.sum(acc.v[COMP][a][b][c]);
    }
    if (lead && rr.last) {
#pragma unroll
        for (int c = 0; c < L; ++c)
#pragma unroll
            for (int b = 0; b < L; ++b)
#pragma unroll
                for (int a = 0; a < L; ++a)
                    if (RegJ<real, L>::used(COMP, a, b, c)) J.add(COMP, a, b, c, acc.v[COMP][a][b][c]);
    }
}

// Kept-node currents of a wave, summed over runs of neighbouring lanes that
// share a reference node (node-major order puts a node's particles side by
// side) and added to LDS by one leader lane per run.  Every lane of the wave
// calls it.  A particle that changed node contributes zero here (its offsets
// and displacement are finite, its charge factor is zeroed) but keeps its
// place in its node's run, so that a node's run is not split in two whose
// leaders would add to the same LDS addresses in one instruction; only
// lanes outside the staged windows break runs.
template <typename real, int M, int TX, int TY, int TZ, int H>
__device__ __forceinline__ void deposit_runs(const Deferred<real> &df, double *sJ) {
    using C = Cfg<real, M, TX, TY, TZ, H>;
    constexpr int L = M + 1;
    const bool inwin = df.keep || df.want;
    RowRuns<real> rr;
    rr.set(inwin ? df.rel : -1 - (int)__lane_id());
    DepW<real, M> DW[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) DW[d].set_kept(df.d0[d], df.D[d]);
    const real coef = df.keep ? df.coef : (real)0;
    const int pk = df.rel;
    const int r0 = (pk & 255) - 8, r1 = ((pk >> 8) & 255) - 8, r2 = ((pk >> 16) & 255) - 8;
    LdsJ<real, C> J{sJ, (r0 + H + C::RL_J) + C::JX * ((r1 + H + C::RL_J) + C::JY * (r2 + H + C::RL_J)), 0};
    J.begin(DW[0].s, DW[1].s, DW[2].s);
    // one component at a time keeps (M+1)^2 M partial sums live
    runs_comp<real, M, 0>(J, DW, coef, rr, inwin);
    runs_comp<real, M, 1>(J, DW, coef, rr, inwin);
    runs_comp<real, M, 2>(J, DW, coef, rr, inwin);
}

// Slots of a block's table of foreign boxes: a tile and the cells its
// particles may drift into before the next sort meet at most 8 boxes of the
// smallest edge (16 cells) that tiles nest in.
constexpr int kForeignSlots = 16;

// Counts one particle whose cell lies outside its tile's box under the box
// that holds the cell (open addressing; a full table leaves the particle
// with the tile's box).
__device__ __forceinline__ void note_foreign(const BoxMap &bm, uint32_t cell, int *sbox, unsigned *scnt,
                                             unsigned &sany) {
    int x, y, z;
    unpack_cell(cell, x, y, z);
    const int b = bm.coarse_box[(x / bm.g[0]) + bm.cg[0] * ((y / bm.g[1]) + bm.cg[1] * (z / bm.g[2]))];
#pragma unroll 1
    for (int k = 0; k < kForeignSlots; ++k) {
        const int slot = (b + k) & (kForeignSlots - 1);
        const int prev = atomicCAS(&sbox[slot], -1, b);
        if (prev == -1 || prev == b) {
            atomicAdd(&scnt[slot], 1u);
            sany = 1;
            return;
        }
    }
}

template <typename real, int M, int TX, int TY, int TZ, int H, bool R>
__global__ __launch_bounds__(512) void k_gpd(GpdArgs<real> A) {
    using C = Cfg<real, M, TX, TY, TZ, H>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    real *sEB = reinterpret_cast<real *>(smem_raw);
    double *sJ = reinterpret_cast<double *>(smem_raw + (size_t)6 * C::NEB * sizeof(real));
    real *qr = reinterpret_cast<real *>(smem_raw + C::lds);           // [7][blockDim.x]
    int *qi = reinterpret_cast<int *>(qr + 7 * blockDim.x);          // [blockDim.x]
    __shared__ unsigned long long sCyc, sRtc;
    __shared__ int sItem[3];
    __shared__ real sSpc[2 * kMaxSpecies];  // per species: q dt / (2 m), -q / dt
    __shared__ int sQn[8];  // queue lengths of the block's waves at the end of an item
    // particles of the item whose cell lies outside the tile's box (they
    // drifted across a box face since the last sort), counted per box
    __shared__ int sFBox[kForeignSlots];
    __shared__ unsigned sFCnt[kForeignSlots];
    __shared__ unsigned sFAny;
    // the field update's early part may share the CUs, and has slack: this
    // kernel's waves take instruction-issue priority over its waves
    __builtin_amdgcn_s_setprio(1);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int nsp = A.nsp;
    const int home = blockIdx.x % kSubQueues;  // blocks are dealt round-robin over the XCDs
    // windows reach at most JX cells; one conditional wrap suffices unless the
    // domain is smaller than a window
    const bool small = A.n[0] < C::JX || A.n[1] < C::JY || A.n[2] < C::JZ;
    int sq = 0;                                // sub-queues already found empty (thread 0)

    // the J window starts clear; each flush clears what it reads
    for (int i = tid; i < 3 * C::NJ; i += nthr) sJ[i] = 0.0;
    if (tid < kMaxSpecies) {
        sSpc[2 * tid] = A.h[tid];
        sSpc[2 * tid + 1] = A.coefq[tid];
    }
    for (int iter = 0;; ++iter) {
        int tile, pbeg, pend;
        if (tid < kForeignSlots) {
            sFBox[tid] = -1;
            sFCnt[tid] = 0;
        }
        if (tid == 0) sFAny = 0;
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
            // the same for every thread: held in scalar registers
            tile = __builtin_amdgcn_readfirstlane(sItem[0]);
            pbeg = __builtin_amdgcn_readfirstlane(sItem[1]);
            pend = __builtin_amdgcn_readfirstlane(sItem[2]);
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
            __syncthreads();  // the table of foreign boxes is clear
        }
        const TileDesc td = A.tiles[tile];
        // the tile's box, for charging each particle's work to the box that
        // holds its cell at the start of the step (wave-uniform)
        const uint32_t box_lo = __builtin_amdgcn_readfirstlane(td.box_lo);
        const uint32_t box_hi = __builtin_amdgcn_readfirstlane(td.box_hi);

        // stage E and B of the tile window (one index computation serves the
        // six components; windows inside the domain need no wrap)
        {
            const int ox = td.x0 - H - C::RL_EB, oy = td.y0 - H - C::RL_EB, oz = td.z0 - H - C::RL_EB;
            const bool inside = ox >= 0 && oy >= 0 && oz >= 0 && ox + C::EX <= A.n[0] && oy + C::EY <= A.n[1] &&
                                oz + C::EZ <= A.n[2];
            const size_t sy = (size_t)A.n[0], sz = (size_t)A.n[0] * A.n[1];
            for (int i0 = 0; i0 < C::NEB; i0 += nthr) {
                const int i = i0 + tid;
                if (i >= C::NEB) continue;
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
                if constexpr (std::is_same<real, float>::value) {
                    // straight from global memory into the window (each
                    // lane's word lands at the wave's base + 4 * lane)
                    const int wbase = i0 + (tid & ~63);
#pragma unroll
                    for (int comp = 0; comp < 6; ++comp)
                        __builtin_amdgcn_global_load_lds((const void *)&A.EB[comp][g], (void *)(sEB + comp * C::NEB + wbase), 4, 0, 0);
                } else {
                    real v[6];
#pragma unroll
                    for (int comp = 0; comp < 6; ++comp) v[comp] = A.EB[comp][g];
#pragma unroll
                    for (int comp = 0; comp < 6; ++comp) sEB[comp * C::NEB + i] = v[comp];
                }
            }
            if constexpr (std::is_same<real, float>::value) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        }
        if (tid == 0) {
            sCyc = 0;
            sRtc = 0;
        }
        __syncthreads();

        const bool timed = A.timer != 0;
        unsigned long long c0 = 0, r0 = 0;
        if (timed) {
            c0 = clock64();
            r0 = wall_clock64();
        }
        const int lane = tid & 63, qslot0 = tid & ~63;
        int qn = 0;  // entries in this wave's queue (wave-uniform)
        {
            // The item's particles, all species together: wave w takes the
            // runs of 64 particles w, w + W, w + 2W, ... (W waves), so that
            // only the item's last run is partly filled and no wave steps
            // through empty runs.  A particle's species follows from the
            // segment bounds inside the tile.
            const int sb = pbeg, se = pend;
            int bnd[kMaxSpecies - 1];  // first particle of species k + 1
#pragma unroll
            for (int k = 0; k < kMaxSpecies - 1; ++k)
                bnd[k] = k + 1 < nsp ? A.segstart[tile * nsp + k + 1] : INT_MAX;
            // the next particle's loads are issued before this one is
            // computed; the trip count is the same for every lane of a wave
            // lanes past the item's end step a zero-weight stand-in, so that
            // every lane runs the same code without branches around it
            const uint32_t origin = pack_cell(td.x0, td.y0, td.z0);
            PState<real> cur;
            if (sb + tid < se) cur.load(A.P, sb + tid);
            else cur.blank(origin);
            cur.settle();
            for (int base = sb + (tid & ~63); base < se; base += nthr) {
                const int p = base + lane;
                PState<real> nxt;
                if (p + nthr < se) nxt.load(A.P, p + nthr);
                else nxt.blank(origin);
                int sp = 0;
#pragma unroll
                for (int k = 0; k < kMaxSpecies - 1; ++k) sp += p >= bnd[k];
                const real hq = sSpc[2 * sp], cq = sSpc[2 * sp + 1];
                Deferred<real> df;
                df.want = false;
                df.keep = false;
                if (timed) {
                    // particles that drifted out of the tile's box since the
                    // last sort are counted under the box that holds them
                    // (the packed bounds are unpacked here, in scalar
                    // registers, rather than kept unpacked across the loop)
                    uint32_t bl = box_lo, bh = box_hi;
                    asm volatile("" : "+s"(bl), "+s"(bh));
                    int cx, cy, cz, lx, ly, lz, hx, hy, hz;
                    unpack_cell(cur.cell, cx, cy, cz);
                    unpack_cell(bl, lx, ly, lz);
                    unpack_cell(bh, hx, hy, hz);
                    // branch-free: one ballot, and a branch only for a wave
                    // that holds such a particle
                    const bool foreign = ((unsigned)(cx - lx) > (unsigned)(hx - lx)) |
                                         ((unsigned)(cy - ly) > (unsigned)(hy - ly)) |
                                         ((unsigned)(cz - lz) > (unsigned)(hz - lz));
                    if (foreign) note_foreign(*A.bmap, cur.cell, sFBox, sFCnt, sFAny);
                }
                PState<real> moved;
                const bool fast = push_staged<real, M, TX, TY, TZ, H, R>(A, cur, td, hq, cq, sEB, sJ, df, moved);
                // a particle beyond the windows is left to the global-path
                // kernel, which runs after this one in the same step
                if (!fast && p < se) A.slowlist[atomicAdd(A.slown, 1u)] = p;
                if constexpr (R) deposit_runs<real, M, TX, TY, TZ, H>(df, sJ);
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
                // the next particle's loads are waited for before this one's
                // stores are issued, so that the wait never covers the stores
                nxt.settle();
                if (p < se && fast) moved.store(A.P, p);
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
        if (timed) {
            unsigned long long c1 = clock64(), r1 = wall_clock64();
            if ((tid & 63) == 0) {
                atomicAdd(&sCyc, c1 - c0);
                atomicAdd(&sRtc, r1 - r0);
            }
        }
        __syncthreads();

        // flush the J window (nonzero entries only)
        {
            const int ox = td.x0 - H - C::RL_J, oy = td.y0 - H - C::RL_J, oz = td.z0 - H - C::RL_J;
            const bool inside = ox >= 0 && oy >= 0 && oz >= 0 && ox + C::JX <= A.n[0] && oy + C::JY <= A.n[1] &&
                                oz + C::JZ <= A.n[2];
            const size_t sy = (size_t)A.n[0], sz = (size_t)A.n[0] * A.n[1];
            // the window's z-planes may now hold current
            if (tid < C::JZ) {
                const int gz = oz + tid;
                A.jdirty[small ? wrap_any(gz, A.n[2]) : wrap_near(gz, A.n[2])] = 1;
            }
            for (int i = tid; i < C::NJ; i += nthr) {
                double dv[3];
#pragma unroll
                for (int comp = 0; comp < 3; ++comp) dv[comp] = sJ[comp * C::NJ + i];
                if (dv[0] == 0.0 && dv[1] == 0.0 && dv[2] == 0.0) continue;
                real v[3];
#pragma unroll
                for (int comp = 0; comp < 3; ++comp) {
                    v[comp] = (real)dv[comp];
                    sJ[comp * C::NJ + i] = 0.0;
                }
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
            if (timed) {
                // the item's cycles are split over the boxes that hold its
                // particles, in proportion to their counts (particles that
                // found no free slot stay with the tile's box)
                const unsigned long long cyc = sCyc, rtc = sRtc;
                unsigned long long cf = 0, rf = 0;
                unsigned nf = 0;
                const unsigned n_item = (unsigned)(pend - pbeg);
                if (sFAny) {
                    const double inv = 1.0 / (double)n_item;
                    for (int k = 0; k < kForeignSlots; ++k) {
                        const int b = sFBox[k];
                        if (b < 0) continue;
                        const unsigned cnt = sFCnt[k];
                        const unsigned long long c = (unsigned long long)((double)cyc * (double)cnt * inv);
                        const unsigned long long r = (unsigned long long)((double)rtc * (double)cnt * inv);
                        if (c) atomicAdd(&A.cycles[b], c);
                        if (r) atomicAdd(&A.rtc[b], r);
                        cf += c;
                        rf += r;
                        nf += cnt;
                    }
                }
                if (nf < n_item) {
                    atomicAdd(&A.cycles[td.box], cyc - cf);
                    atomicAdd(&A.rtc[td.box], rtc - rf);
                }
            }
        }
        __syncthreads();
    }
}

// The global path as a kernel of its own, so that its registers do not add
// to the tile kernel's: the particles listed in slowlist[0, slown[0]) (left
// by the tile kernel, whose windows they have left), or particles [0, n)
// with no list (staging off).  Each particle's work is charged to the box of
// its cell at the start of the step, its wave's clock split evenly over the
// wave's particles.  The last block to finish adds the count to the running
// total of global-path particles and clears the list for the next step.
template <typename real, int M>
__global__ __launch_bounds__(256) void k_gpd_global(GpdArgs<real> A, int n) {
    __shared__ unsigned sN;
    if (threadIdx.x == 0) sN = A.slowlist ? A.slown[0] : (unsigned)n;
    __syncthreads();
    const int cnt = (int)sN;
    const bool timed = A.timer != 0;
    const int stride = gridDim.x * blockDim.x, lane = (int)(threadIdx.x & 63u);
    // the trip count is the same for every lane of a wave (clock reads are
    // wave-wide); the next particle's loads are issued before this one is
    // computed
    int base = blockIdx.x * blockDim.x + (int)(threadIdx.x & ~63u);
    PState<real> cur;
    int p = 0, sp = 0;
    bool live = base + lane < cnt;
    if (live) {
        p = A.slowlist ? A.slowlist[base + lane] : base + lane;
        cur.load(A.P, p);
        sp = A.P.sp[p];
    } else {
        cur.blank(0);
    }
    for (; base < cnt; base += stride) {
        const int kn = base + stride + lane;
        const bool live_n = kn < cnt;
        PState<real> nxt;
        int pn = 0, spn = 0;
        if (live_n) {
            pn = A.slowlist ? A.slowlist[kn] : kn;
            nxt.load(A.P, pn);
            spn = A.P.sp[pn];
        } else {
            nxt.blank(0);
        }
        unsigned long long c0 = 0, r0 = 0;
        if (timed) {
            c0 = clock64();
            r0 = wall_clock64();
        }
        int box = 0;
        if (live) {
            int x, y, z;
            unpack_cell(cur.cell, x, y, z);
            const BoxMap &bm = *A.bmap;
            box = bm.coarse_box[(x / bm.g[0]) + bm.cg[0] * ((y / bm.g[1]) + bm.cg[1] * (z / bm.g[2]))];
            PState<real> moved;
            push_global<real, M>(A, cur, A.h[sp], A.coefq[sp], moved);
            moved.store(A.P, p);
        }
        const bool was_live = live;
        cur = nxt;
        p = pn;
        sp = spn;
        live = live_n;
        if (timed && was_live) {
            const unsigned long long c1 = clock64(), r1 = wall_clock64();
            const unsigned long long nl = (unsigned long long)__popcll(__ballot(1));
            atomicAdd(&A.cycles[box], (c1 - c0) / nl);
            atomicAdd(&A.rtc[box], (r1 - r0) / nl);
        }
    }
    if (!A.slowlist) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && cnt > 0) atomicAdd(A.slow, (unsigned)cnt);
        return;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(A.slown + 1, 1u) == gridDim.x - 1) {
            if (cnt > 0) atomicAdd(A.slow, (unsigned)cnt);
            A.slown[0] = 0;
            A.slown[1] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Host launcher
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

// Kernel arguments from the precision-erased launch description.
template <typename real>
static GpdArgs<real> gpd_args_of(const GpdLaunch &L) {
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
    A.bmap = L.bmap;
    A.slow = L.slow;
    A.slowlist = L.slowlist;
    A.slown = L.slown;
    A.jdirty = L.jdirty;
    A.mode = L.mode;
    A.timer = L.timer;
    A.tile_base = L.tile_base;
    A.species_only = L.species_only;
    A.queue = L.queue;
    A.queue_bounds = L.queue_bounds;
    A.queue_head = L.queue_head;
    return A;
}

// Table of compiled gather-push-deposit variants.
template <typename real, int M, int TX, int TY, int TZ, int H, bool R>
static hipError_t gpd_one(const GpdLaunch &L, hipStream_t st) {
    using C = Cfg<real, M, TX, TY, TZ, H>;
    auto kern = k_gpd<real, M, TX, TY, TZ, H, R>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(C::lds + 512 * C::qslot));
        if (e != hipSuccess) return e;
        attr = true;
    }
    if (L.block != 256 && L.block != 384 && L.block != 512) return hipErrorInvalidValue;
    if (L.regs_out) {
        hipFuncAttributes fa;
        hipError_t e = hipFuncGetAttributes(&fa, (const void *)kern);
        if (e != hipSuccess) return e;
        *L.regs_out = fa.numRegs;
    }
    GpdArgs<real> A = gpd_args_of<real>(L);
    if (L.grid == 0) return hipSuccess;
    kern<<<L.grid, L.block, C::lds + (size_t)L.block * C::qslot, st>>>(A);
    return hipGetLastError();
}

template <typename real, int M, bool R>
static hipError_t gpd_tile_r(const GpdLaunch &L, hipStream_t st) {
    const int *T = L.tile;
    if (L.halo != 1) return hipErrorInvalidValue;
    if (T[0] == 8 && T[1] == 8 && T[2] == 8) return gpd_one<real, M, 8, 8, 8, 1, R>(L, st);
    if (T[0] == 8 && T[1] == 8 && T[2] == 4) return gpd_one<real, M, 8, 8, 4, 1, R>(L, st);
    if (T[0] == 8 && T[1] == 4 && T[2] == 4) return gpd_one<real, M, 8, 4, 4, 1, R>(L, st);
    if (T[0] == 4 && T[1] == 4 && T[2] == 4) return gpd_one<real, M, 4, 4, 4, 1, R>(L, st);
    return hipErrorInvalidValue;
}

template <typename real, int M>
hipError_t gpd_tile(const GpdLaunch &L, hipStream_t st) {
    return L.run_sum ? gpd_tile_r<real, M, true>(L, st) : gpd_tile_r<real, M, false>(L, st);
}

// The global-path kernel: over the tile kernels' list (n < 0), or over
// particles [0, n) with no list.
template <typename real, int M>
hipError_t gpd_global(const GpdLaunch &L, int n, unsigned grid, hipStream_t st) {
    GpdArgs<real> A = gpd_args_of<real>(L);
    if (n >= 0) A.slowlist = nullptr;
    if (grid == 0) return hipSuccess;
    k_gpd_global<real, M><<<grid, 256, 0, st>>>(A, n < 0 ? 0 : n);
    return hipGetLastError();
}

}  // namespace pb
