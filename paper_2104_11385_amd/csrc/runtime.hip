// Host runtime of libpicbal: context, initialisation, the step loop (sort
// schedule, launch modes, hipGraph replay), per-box costs and counts, state
// access and kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include <map>

#include "kernels.hpp"
#include "runtime.hpp"

using namespace pb;

namespace {

thread_local std::string g_init_error;

// Autotuner results, shared by contexts of the same workload signature.
std::map<std::string, pic_tuning> g_tune_cache;

// LDS of one gfx950 compute unit.
constexpr size_t kLdsPerCu = 160 * 1024;

// Blocks of the gather-push-deposit kernel that the LDS of one CU holds at
// once (1 to 4).
int resident_blocks(int prec, int order, const int tile[3], int block) {
    size_t lds = gpd_lds_bytes(prec, order, tile, 1, block);
    int n = lds ? (int)(kLdsPerCu / lds) : 1;
    return n < 1 ? 1 : (n > 4 ? 4 : n);
}

const char *status_text(int code) {
    switch (code) {
    case PIC_OK: return "ok";
    case PIC_EINVAL: return "invalid argument";
    case PIC_ENOMEM: return "out of memory";
    case PIC_EDEVICE: return "HIP device error";
    case PIC_ECFL: return "time step violates the 3D Courant condition (dt >= 1/sqrt(3))";
    case PIC_ECAPACITY: return "particle capacity exceeded";
    case PIC_ESTATE: return "invalid state for this call";
    case PIC_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
    }
}

int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a < 0 ? -a : a;
}

}  // namespace

// ---------------------------------------------------------------------------
// pic_ctx helpers
// ---------------------------------------------------------------------------

int pic_ctx::fail(int code, const std::string &msg) {
    err = msg;
    if (code == PIC_EDEVICE) sticky = PIC_EDEVICE;
    return code;
}

int pic_ctx::hip_fail(hipError_t e, const char *what) {
    return fail(PIC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPC(expr)                                      \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

int pic_ctx::dalloc(void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PIC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    allocs.push_back(*p);
    return PIC_OK;
}

Geom pic_ctx::geom() const {
    Geom G;
    for (int d = 0; d < 3; ++d) {
        G.n[d] = n[d];
        G.T[d] = tun.tile[d];
        G.g[d] = g[d];
        G.cg[d] = cg[d];
    }
    G.Tvol = tun.tile[0] * tun.tile[1] * tun.tile[2];
    G.coarse_box = d_coarse_box;
    G.box_lo = d_box_lo;
    G.box_nt = d_box_nt;
    G.box_tile_off = d_box_tile_off;
    G.nsp = nsp;
    G.order = order;
    return G;
}

void pic_ctx::drop_graphs() {
    for (auto &plane : gexec)
        for (auto &row : plane)
            for (auto &e : row)
                if (e) {
                    (void)hipGraphExecDestroy(e);
                    e = nullptr;
                }
}

// Builds the tile table for the current tuning and (re)allocates the sort
// scratch and queue that depend on it.
int pic_ctx::build_tiles() {
    const int *T = tun.tile;
    std::vector<int> nt(3 * nb), off(nb + 1, 0);
    std::vector<TileDesc> tiles;
    for (int b = 0; b < nb; ++b) {
        int ntb = 1;
        for (int d = 0; d < 3; ++d) {
            int e = boxes[b].hi[d] - boxes[b].lo[d];
            if (e % T[d]) return fail(PIC_EUNSUPPORTED, "tile edge does not divide a box edge");
            nt[3 * b + d] = e / T[d];
            ntb *= e / T[d];
        }
        off[b + 1] = off[b] + ntb;
        for (int tz = 0; tz < nt[3 * b + 2]; ++tz)
            for (int ty = 0; ty < nt[3 * b + 1]; ++ty)
                for (int tx = 0; tx < nt[3 * b]; ++tx)
                    tiles.push_back({boxes[b].lo[0] + tx * T[0], boxes[b].lo[1] + ty * T[1],
                                     boxes[b].lo[2] + tz * T[2], b,
                                     pack_cell(boxes[b].lo[0], boxes[b].lo[1], boxes[b].lo[2]),
                                     pack_cell(boxes[b].hi[0] - 1, boxes[b].hi[1] - 1, boxes[b].hi[2] - 1)});
    }
    ntiles = off[nb];
    h_box_tile_off = off;
    free_tile_buffers();
    int rc;
    if ((rc = dalloc((void **)&d_box_nt, sizeof(int) * 3 * nb))) return rc;
    tile_allocs.push_back(d_box_nt);
    if ((rc = dalloc((void **)&d_box_tile_off, sizeof(int) * (nb + 1)))) return rc;
    tile_allocs.push_back(d_box_tile_off);
    if ((rc = dalloc((void **)&d_tiles, sizeof(TileDesc) * ntiles))) return rc;
    tile_allocs.push_back(d_tiles);
    HIPC(hipMemcpy(d_box_nt, nt.data(), sizeof(int) * 3 * nb, hipMemcpyHostToDevice));
    HIPC(hipMemcpy(d_box_tile_off, off.data(), sizeof(int) * (nb + 1), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(d_tiles, tiles.data(), sizeof(TileDesc) * ntiles, hipMemcpyHostToDevice));

    int Tvol = T[0] * T[1] * T[2];
    W.nseg = ntiles * nsp;
    size_t ncell = (size_t)W.nseg * Tvol;
    if ((rc = dalloc((void **)&W.cellcnt, sizeof(uint32_t) * ncell))) return rc;
    tile_allocs.push_back(W.cellcnt);
    if ((rc = dalloc((void **)&W.cellstart, sizeof(uint32_t) * ncell))) return rc;
    tile_allocs.push_back(W.cellstart);
    if ((rc = dalloc((void **)&W.segtot, sizeof(int) * W.nseg))) return rc;
    tile_allocs.push_back(W.segtot);
    if ((rc = dalloc((void **)&W.segstart, sizeof(int) * (W.nseg + 1)))) return rc;
    tile_allocs.push_back(W.segstart);
    size_t nb1 = (size_t)W.nseg / 1024 + 2;
    if ((rc = dalloc((void **)&W.bsum, sizeof(int) * nb1))) return rc;
    tile_allocs.push_back(W.bsum);
    if ((rc = dalloc((void **)&W.boff, sizeof(int) * (nb1 + 1)))) return rc;
    tile_allocs.push_back(W.boff);
    int chunk = std::max(64, tun.chunk);
    size_t qmax = (size_t)ntiles + (size_t)(cap / chunk) + 1;
    if ((rc = dalloc((void **)&Q.queue, sizeof(int4) * qmax))) return rc;
    tile_allocs.push_back(Q.queue);
    return PIC_OK;
}

void pic_ctx::free_tile_buffers() {
    for (void *p : tile_allocs) {
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) allocs.erase(it);
        (void)hipFree(p);
    }
    tile_allocs.clear();
}

int pic_ctx::sort_now() {
    int next = 1 - pcur;
    HIPC(launch_sort(prec, P[pcur], P[next], (int)np, geom(), W, tun.run_sum != 0, st));
    pcur = next;
    steps_since_sort = 0;
    int chunk = std::max(64, tun.chunk);
    HIPC(launch_queue(W.segstart, ntiles, nsp, chunk, Q, st));
    return PIC_OK;
}

GpdLaunch pic_ctx::gpd_args() const {
    GpdLaunch L;
    L.P = P[pcur];
    L.segstart = W.segstart;
    L.tiles = d_tiles;
    for (int c = 0; c < 3; ++c) {
        L.EB[c] = Eb[jcur][c];
        L.EB[3 + c] = Bb[jcur][c];
        L.J[c] = Jb[jcur][c];
    }
    for (int d = 0; d < 3; ++d) {
        L.n[d] = n[d];
        L.tile[d] = tun.tile[d];
    }
    L.nsp = nsp;
    L.dt = dt;
    for (int d = 0; d < 3; ++d) L.bext[d] = bext[d];
    for (int s = 0; s < kMaxSpecies; ++s) {
        L.h[s] = s < nsp ? sp[s].q * dt / (2.0 * sp[s].m) : 0.0;
        L.coefq[s] = s < nsp ? -sp[s].q / dt : 0.0;
    }
    L.cycles = d_cycles;
    L.rtc = d_rtc;
    L.bmap = d_bmap;
    L.slow = d_slow;
    // the sort's rank array is idle between sorts
    L.slowlist = (int *)W.rank;
    L.slown = d_slown;
    L.jdirty = d_jdirty[jcur];
    L.mode = mode;
    L.timer = cost_timer ? 1 : 0;
    L.staged = staged ? 1 : 0;
    L.tile_base = 0;
    L.species_only = -1;
    L.queue = Q.queue;
    L.queue_bounds = Q.queue_bounds;
    L.queue_head = Q.queue_head;
    L.halo = tun.halo;
    L.run_sum = tun.run_sum;
    L.block = (unsigned)tun.block;
    L.grid = 0;
    L.regs_out = nullptr;
    return L;
}

int pic_ctx::time_begin(int kind) {
    if (!timing || capturing) return PIC_OK;
    hipEvent_t a, b;
    HIPC(hipEventCreate(&a));
    HIPC(hipEventCreate(&b));
    HIPC(hipEventRecord(a, st));
    ev_pending = {a, b};
    ev_kind = kind;
    return PIC_OK;
}

int pic_ctx::time_end() {
    if (!timing || capturing) return PIC_OK;
    HIPC(hipEventRecord(ev_pending.second, st));
    events[ev_kind].push_back(ev_pending);
    return PIC_OK;
}

// Queues one step (gather-push-deposit + Yee) on the stream.
int pic_ctx::enqueue_step() {
    GpdLaunch L = gpd_args();
    int rc;
    // the field update of the planes that no deposit of this step reaches
    // runs on the second stream beside the particle kernels (it needs what
    // the previous step left: E^n, the half-step B and the current flags)
    YeeBuffers Y = yee_buffers();
    const bool split = tun.field_overlap != 0;
    // the early part takes few blocks per CU, so that it fits beside the
    // particle kernel's blocks whichever is dispatched first: one with at
    // least as many particles as cells (the particle kernel then outlasts it
    // by far; on the 256^3 slab 0.6% faster steps than with two), two with
    // at least half as many; with fewer the particle kernel is the shorter
    // branch (about 50 ps per particle against 27 ps per cell for two blocks
    // per CU) and the early part takes eight
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    const unsigned yee_early = (unsigned)((np >= cells ? 1 : (2 * np >= cells ? 2 : 8)) * n_cu);
    // the rest: 64 blocks per CU, or enough that no block takes more than
    // eight units (row segments) of the plane list; blocks that step through
    // more units lose the neighbour planes they share from the caches
    // (512^3, all planes after the particle kernel: 3.06 ms per update with
    // 32 units per block, 2.70 with 8; 256^3: 0.26 ms with 4)
    const size_t units = ((size_t)n[0] * n[1] + 255) / 256 * (size_t)n[2];
    const unsigned yee_grid = (unsigned)std::max<size_t>((size_t)64 * n_cu, (units + 7) / 8);
    // (the same one-block kernel rewinds the persistent queue's heads)
    HIPC(launch_yee_class(Y, n[2], split, mode == MODE_PERSISTENT && staged ? Q.queue_head : nullptr, st));
    if (split) {
        HIPC(hipEventRecord(ev_fork, st));
        HIPC(hipStreamWaitEvent(st2, ev_fork, 0));
        HIPC(launch_yee(prec, Y, n, dt, 0, yee_early, st2));
        HIPC(hipEventRecord(ev_join, st2));
    }
    if ((rc = time_begin(0))) return rc;
    if (!staged) {
        // reference path: every particle through the global arrays
        const unsigned g = (unsigned)std::min<int64_t>((np + 255) / 256, (int64_t)n_cu * 8);
        HIPC(launch_gpd_global(prec, order, L, (int)np, g, st));
    } else if (mode == MODE_PER_BOX) {
        for (int b = 0; b < nb; ++b)
            for (int s = 0; s < nsp; ++s) {
                L.tile_base = h_box_tile_off[b];
                L.species_only = s;
                L.grid = (unsigned)(h_box_tile_off[b + 1] - h_box_tile_off[b]);
                HIPC(launch_gpd(prec, order, L, st));
            }
    } else if (mode == MODE_BATCHED) {
        L.grid = (unsigned)ntiles;
        HIPC(launch_gpd(prec, order, L, st));
    } else {
        L.grid = (unsigned)(n_cu * std::max(1, tun.blocks_per_cu));
        HIPC(launch_gpd(prec, order, L, st));
    }
    // the particles the tile kernels left to the global path (rare: those
    // that drifted beyond their tile's windows since the last sort)
    if (staged) HIPC(launch_gpd_global(prec, order, L, -1, (unsigned)n_cu, st));
    if ((rc = time_end())) return rc;
    if (split) HIPC(hipStreamWaitEvent(st, ev_join, 0));
    if ((rc = time_begin(1))) return rc;
    HIPC(launch_yee(prec, Y, n, dt, 1, yee_grid, st));
    if ((rc = time_end())) return rc;
    return PIC_OK;
}

// Marks every z-plane of both J buffers as possibly nonzero (after J was
// written from outside the step).
int pic_ctx::mark_j_dirty() {
    for (int b = 0; b < 2; ++b)
        if (launch_fill_u32((uint32_t *)d_jdirty[b], (size_t)n[2], st, 1u) != hipSuccess) return PIC_EDEVICE;
    return PIC_OK;
}

YeeBuffers pic_ctx::yee_buffers() const {
    YeeBuffers Y;
    for (int c = 0; c < 3; ++c) {
        Y.E[c] = Eb[jcur][c];
        Y.B[c] = Bb[jcur][c];
        Y.J[c] = Jb[jcur][c];
        Y.X[c] = Xb[c];
        Y.Eo[c] = Eb[1 - jcur][c];
        Y.Bo[c] = Bb[1 - jcur][c];
        Y.Z[c] = Jb[1 - jcur][c];
    }
    Y.jdirty = d_jdirty[jcur];
    Y.zdirty = d_jdirty[1 - jcur];
    Y.lists = d_ylists;
    return Y;
}

// Computes the half-step B from the current fields (eagerly, outside any
// captured graph) when it is not current.
int pic_ctx::yee_half() {
    if (xvalid) return PIC_OK;
    int rc;
    if ((rc = time_begin(1))) return rc;
    YeeBuffers Y = yee_buffers();
    HIPC(launch_yee_half(prec, Y, n, dt, st));
    if ((rc = time_end())) return rc;
    xvalid = true;
    return PIC_OK;
}

// In graph mode every step is one graph launch: a step that starts with the
// periodic particle sort (and work-queue rebuild) replays a graph captured
// with the sort in it.
int pic_ctx::step(int nsteps) {
    for (int i = 0; i < nsteps; ++i) {
        if (int rc = yee_half()) return rc;
        const bool do_sort = steps_since_sort >= std::max(1, tun.sort_interval);
        if (use_graph) {
            hipGraphExec_t &ge = gexec[do_sort ? 1 : 0][jcur][pcur];
            if (!ge) {
                hipGraph_t gr;
                capturing = true;
                HIPC(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                int rc = do_sort ? sort_now() : PIC_OK;  // flips pcur
                if (!rc) rc = enqueue_step();
                hipError_t e2 = hipStreamEndCapture(st, &gr);
                capturing = false;
                if (rc) return rc;
                HIPC(e2);
                HIPC(hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0));
                HIPC(hipGraphDestroy(gr));
            } else if (do_sort) {
                pcur = 1 - pcur;
                steps_since_sort = 0;
            }
            HIPC(hipGraphLaunch(ge, st));
        } else {
            int rc;
            if (do_sort) {
                if ((rc = time_begin(2))) return rc;
                if ((rc = sort_now())) return rc;
                if ((rc = time_end())) return rc;
            }
            if ((rc = enqueue_step())) return rc;
        }
        jcur = 1 - jcur;
        ++steps_since_sort;
        ++step_no;
    }
    return PIC_OK;
}

// Host <-> device particle state (double global positions on the host).
int pic_ctx::download(std::vector<uint32_t> &cell, std::vector<double> f[3], std::vector<double> u[3],
                      std::vector<double> &w, std::vector<int64_t> &id, std::vector<uint8_t> &spv) {
    HIPC(hipStreamSynchronize(st));
    size_t m = (size_t)np;
    cell.resize(m);
    id.resize(m);
    spv.resize(m);
    w.resize(m);
    for (int d = 0; d < 3; ++d) {
        f[d].resize(m);
        u[d].resize(m);
    }
    if (m == 0) return PIC_OK;
    const ParticlesRaw &R = P[pcur];
    HIPC(hipMemcpy(cell.data(), R.cell, 4 * m, hipMemcpyDeviceToHost));
    HIPC(hipMemcpy(id.data(), R.id, 8 * m, hipMemcpyDeviceToHost));
    HIPC(hipMemcpy(spv.data(), R.sp, m, hipMemcpyDeviceToHost));
    auto get = [&](std::vector<double> &dst, const void *src) -> int {
        if (prec == 8) {
            HIPC(hipMemcpy(dst.data(), src, 8 * m, hipMemcpyDeviceToHost));
        } else {
            std::vector<float> tmp(m);
            HIPC(hipMemcpy(tmp.data(), src, 4 * m, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < m; ++i) dst[i] = tmp[i];
        }
        return PIC_OK;
    };
    int rc;
    for (int d = 0; d < 3; ++d) {
        if ((rc = get(f[d], R.f[d]))) return rc;
        if ((rc = get(u[d], R.u[d]))) return rc;
    }
    return get(w, R.w);
}

int pic_ctx::upload(const std::vector<uint32_t> &cell, const std::vector<double> f[3],
                    const std::vector<double> u[3], const std::vector<double> &w, const std::vector<int64_t> &id,
                    const std::vector<uint8_t> &spv) {
    size_t m = cell.size();
    if ((int64_t)m > cap) return fail(PIC_ECAPACITY, "particle capacity exceeded");
    HIPC(hipStreamSynchronize(st));
    np = (int64_t)m;
    const ParticlesRaw &R = P[pcur];
    if (m) {
        HIPC(hipMemcpy(R.cell, cell.data(), 4 * m, hipMemcpyHostToDevice));
        HIPC(hipMemcpy(R.id, id.data(), 8 * m, hipMemcpyHostToDevice));
        HIPC(hipMemcpy(R.sp, spv.data(), m, hipMemcpyHostToDevice));
    }
    auto put = [&](void *dst, const std::vector<double> &src) -> int {
        if (!m) return PIC_OK;
        if (prec == 8) {
            HIPC(hipMemcpy(dst, src.data(), 8 * m, hipMemcpyHostToDevice));
        } else {
            std::vector<float> tmp(m);
            for (size_t i = 0; i < m; ++i) tmp[i] = (float)src[i];
            HIPC(hipMemcpy(dst, tmp.data(), 4 * m, hipMemcpyHostToDevice));
        }
        return PIC_OK;
    };
    int rc;
    for (int d = 0; d < 3; ++d) {
        if ((rc = put(R.f[d], f[d]))) return rc;
        if ((rc = put(R.u[d], u[d]))) return rc;
    }
    if ((rc = put(R.w, w))) return rc;
    drop_graphs();
    // new positions: every plane of J may be reached by the next deposit
    if (mark_j_dirty()) return fail(PIC_EDEVICE, "J plane flags");
    return sort_now();
}

pic_ctx::~pic_ctx() {
    if (!allocs.empty() || own_stream) (void)hipStreamSynchronize(st);
    drop_graphs();
    for (int k = 0; k < 4; ++k)
        for (auto &e : events[k]) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    mlp_release();
    if (st2) (void)hipStreamSynchronize(st2);
    for (void *p : allocs) (void)hipFree(p);
    if (own_stream) (void)hipStreamDestroy(st);
    if (st2) (void)hipStreamDestroy(st2);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
}

// ---------------------------------------------------------------------------
// C API
// ---------------------------------------------------------------------------

extern "C" {

PIC_API const char *pic_strerror(int code) { return status_text(code); }

PIC_API const char *pic_last_error(pic_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

static int init_fail(pic_ctx *c, int code, const std::string &msg) {
    g_init_error = msg.empty() && c ? c->err : msg;
    delete c;
    return code;
}

PIC_API int pic_init(const pic_grid_desc *grid, const pic_box *boxes, int32_t n_boxes,
                     const pic_species_desc *species, int32_t n_species, void *hip_stream, pic_ctx **out) {
    if (!grid || !boxes || !out || n_boxes < 1 || n_species < 1 || n_species > kMaxSpecies || (!species))
        return init_fail(nullptr, PIC_EINVAL, "null pointer or bad box/species count");
    *out = nullptr;
    const int lim[3] = {2048, 2048, 1024};
    for (int d = 0; d < 3; ++d)
        if (grid->n_cells[d] < 1 || grid->n_cells[d] > lim[d])
            return init_fail(nullptr, PIC_EINVAL, "domain size out of range");
    if (grid->shape_order < 1 || grid->shape_order > 3)
        return init_fail(nullptr, PIC_EINVAL, "shape_order must be 1, 2 or 3");
    if (grid->precision != PIC_FP32 && grid->precision != PIC_FP64)
        return init_fail(nullptr, PIC_EINVAL, "precision must be PIC_FP32 or PIC_FP64");
    if (!(grid->dt > 0.0)) return init_fail(nullptr, PIC_EINVAL, "dt must be positive");
    if (!(grid->dt < 1.0 / std::sqrt(3.0))) return init_fail(nullptr, PIC_ECFL, "dt >= 1/sqrt(3)");

    pic_ctx *c = new pic_ctx();
    for (int d = 0; d < 3; ++d) {
        c->n[d] = grid->n_cells[d];
        c->bext[d] = grid->b_ext[d];
    }
    c->dt = grid->dt;
    c->order = grid->shape_order;
    c->prec = grid->precision;
    c->seed = grid->seed;
    c->wp = grid->w_particle;
    c->wc = grid->w_cell;
    c->nb = n_boxes;
    c->boxes.assign(boxes, boxes + n_boxes);
    c->nsp = n_species;

    // boxes must tile the domain: inside, non-empty, no overlap, no gap
    int64_t vol = 0;
    for (int b = 0; b < n_boxes; ++b)
        for (int d = 0; d < 3; ++d) {
            if (boxes[b].lo[d] < 0 || boxes[b].hi[d] > c->n[d] || boxes[b].hi[d] <= boxes[b].lo[d])
                return init_fail(c, PIC_EINVAL, "box outside the domain or empty");
        }
    for (int d = 0; d < 3; ++d) {
        int64_t g = c->n[d];
        for (int b = 0; b < n_boxes; ++b) g = gcd64(gcd64(g, boxes[b].lo[d]), boxes[b].hi[d]);
        c->g[d] = (int)g;
        c->cg[d] = c->n[d] / (int)g;
    }
    std::vector<int> coarse((size_t)c->cg[0] * c->cg[1] * c->cg[2], -1);
    for (int b = 0; b < n_boxes; ++b) {
        vol += (int64_t)(boxes[b].hi[0] - boxes[b].lo[0]) * (boxes[b].hi[1] - boxes[b].lo[1]) *
               (boxes[b].hi[2] - boxes[b].lo[2]);
        for (int z = boxes[b].lo[2] / c->g[2]; z < boxes[b].hi[2] / c->g[2]; ++z)
            for (int y = boxes[b].lo[1] / c->g[1]; y < boxes[b].hi[1] / c->g[1]; ++y)
                for (int x = boxes[b].lo[0] / c->g[0]; x < boxes[b].hi[0] / c->g[0]; ++x) {
                    int &o = coarse[x + (size_t)c->cg[0] * (y + (size_t)c->cg[1] * z)];
                    if (o >= 0) return init_fail(c, PIC_EINVAL, "boxes overlap");
                    o = b;
                }
    }
    if (vol != (int64_t)c->n[0] * c->n[1] * c->n[2]) return init_fail(c, PIC_EINVAL, "boxes leave a gap");

    // species and particle counts
    std::vector<int64_t> box_cells(n_boxes);
    for (int b = 0; b < n_boxes; ++b)
        box_cells[b] = (int64_t)(boxes[b].hi[0] - boxes[b].lo[0]) * (boxes[b].hi[1] - boxes[b].lo[1]) *
                       (boxes[b].hi[2] - boxes[b].lo[2]);
    int64_t total = 0, totcap = 0;
    for (int s = 0; s < n_species; ++s) {
        const pic_species_desc &S = species[s];
        if (!(S.mass > 0.0)) return init_fail(c, PIC_EINVAL, "species mass must be positive");
        c->sp[s].q = S.charge;
        c->sp[s].m = S.mass;
        c->sp[s].density = S.density;
        c->sp[s].mode = S.load_mode;
        int64_t cnt = 0;
        if (S.load_mode == 1) {
            if (S.ppc < 1) return init_fail(c, PIC_EINVAL, "ppc must be >= 1");
            int64_t cells = 1;
            for (int d = 0; d < 3; ++d) {
                if (S.region_lo[d] < 0 || S.region_hi[d] > c->n[d] || S.region_hi[d] <= S.region_lo[d])
                    return init_fail(c, PIC_EINVAL, "loading region outside the domain or empty");
                cells *= S.region_hi[d] - S.region_lo[d];
            }
            cnt = cells * S.ppc;
        } else if (S.load_mode == 2) {
            if (!S.box_ppc) return init_fail(c, PIC_EINVAL, "box_ppc missing");
            c->sp[s].box_ppc.assign(S.box_ppc, S.box_ppc + n_boxes);
            for (int b = 0; b < n_boxes; ++b) {
                if (S.box_ppc[b] < 0) return init_fail(c, PIC_EINVAL, "negative box ppc");
                cnt += box_cells[b] * S.box_ppc[b];
            }
        } else if (S.load_mode != 0) {
            return init_fail(c, PIC_EINVAL, "load_mode must be 0, 1 or 2");
        }
        c->sp[s].count = cnt;
        c->sp[s].cap = std::max<int64_t>(cnt, S.capacity);
        total += cnt;
        totcap += c->sp[s].cap;
    }
    if (totcap > (int64_t)INT32_MAX - 1) return init_fail(c, PIC_EUNSUPPORTED, "more than 2^31-1 particles");
    c->np = total;
    c->cap = std::max<int64_t>(totcap, 1);

    // device
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, 0) != hipSuccess || hipGetDevice(&c->dev) != hipSuccess)
        return init_fail(c, PIC_EDEVICE, "no HIP device");
    (void)hipGetDeviceProperties(&prop, c->dev);
    c->n_cu = prop.multiProcessorCount;
    {
        std::string serr;
        if (int rc0 = pb_noalloc_setup(c->dev, serr)) return init_fail(c, rc0, serr);
    }
    if (hip_stream) {
        c->st = (hipStream_t)hip_stream;
        c->own_stream = false;
    } else {
        if (hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) != hipSuccess)
            return init_fail(c, PIC_EDEVICE, "hipStreamCreate failed");
        c->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&c->st2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess)
        return init_fail(c, PIC_EDEVICE, "stream or event creation failed");

    // default tuning: 8x4x4 tiles in two 512-thread blocks per CU where the
    // tile divides every box edge, two blocks' LDS fit a CU and the kernel's
    // registers allow the four waves per SIMD that makes (the FP32 kernels of
    // orders 1 and 2: 98-110 VGPRs; on the 256^3 slab 1.19 ms per launch
    // against 1.35 ms for 4x4x4 tiles in three 256-thread blocks).  Else the
    // largest compiled tile that divides every box edge and leaves room for
    // three resident 256-thread blocks per CU, else for two, else for one; as
    // many persistent blocks per CU as the LDS holds
    c->tun.halo = 1;
    c->tun.block = 256;
    c->tun.chunk = 4096;
    c->tun.sort_interval = 20;
    c->tun.run_sum = 1;
    c->tun.field_overlap = 1;
    const int cand[4][3] = {{8, 4, 4}, {4, 4, 4}, {8, 8, 4}, {8, 8, 8}};
    bool chosen = false;
    for (size_t limit : {(size_t)kLdsPerCu / 3, (size_t)kLdsPerCu / 2, (size_t)kLdsPerCu}) {
        for (auto &t : cand) {
            if (chosen) break;
            bool ok = true;
            for (int b = 0; b < n_boxes && ok; ++b)
                for (int d = 0; d < 3; ++d)
                    if ((boxes[b].hi[d] - boxes[b].lo[d]) % t[d]) ok = false;
            if (!ok || gpd_lds_bytes(c->prec, c->order, t, 1, 256) > limit) continue;
            std::memcpy(c->tun.tile, t, sizeof(int) * 3);
            chosen = true;
        }
    }
    if (!chosen) return init_fail(c, PIC_EUNSUPPORTED, "no compiled tile divides every box edge and fits the LDS");
    c->tun.blocks_per_cu = resident_blocks(c->prec, c->order, c->tun.tile, 256);
    {
        const int t4[3] = {8, 4, 4};
        bool ok = gpd_lds_bytes(c->prec, c->order, t4, 1, 512) <= (size_t)kLdsPerCu / 2;
        for (int b = 0; b < n_boxes && ok; ++b)
            for (int d = 0; d < 3; ++d)
                if ((boxes[b].hi[d] - boxes[b].lo[d]) % t4[d]) ok = false;
        int regs = 0;
        if (ok) {
            GpdLaunch q{};
            std::memcpy(q.tile, t4, sizeof(int) * 3);
            q.halo = 1;
            q.run_sum = 1;
            q.block = 512;
            q.grid = 0;
            q.regs_out = &regs;
            ok = launch_gpd(c->prec, c->order, q, c->st) == hipSuccess && regs > 0 && 4 * ((regs + 7) / 8 * 8) <= 512;
        }
        if (ok) {
            std::memcpy(c->tun.tile, t4, sizeof(int) * 3);
            c->tun.block = 512;
            c->tun.blocks_per_cu = 2;
        }
    }

    int rc;
    size_t N = (size_t)c->n[0] * c->n[1] * c->n[2];
    size_t fb = N * (size_t)c->prec;
    for (int k = 0; k < 3; ++k) {
        if ((rc = c->dalloc(&c->Eb[0][k], fb)) || (rc = c->dalloc(&c->Bb[0][k], fb)) ||
            (rc = c->dalloc(&c->Eb[1][k], fb)) || (rc = c->dalloc(&c->Bb[1][k], fb)) ||
            (rc = c->dalloc(&c->Jb[0][k], fb)) || (rc = c->dalloc(&c->Jb[1][k], fb)) ||
            (rc = c->dalloc(&c->Xb[k], fb)))
            return init_fail(c, rc, "");
    }
    for (int b = 0; b < 2; ++b) {
        ParticlesRaw &R = c->P[b];
        size_t m = (size_t)c->cap;
        if ((rc = c->dalloc((void **)&R.cell, 4 * m)) || (rc = c->dalloc((void **)&R.id, 8 * m)) ||
            (rc = c->dalloc((void **)&R.sp, m)) || (rc = c->dalloc(&R.w, m * c->prec)))
            return init_fail(c, rc, "");
        for (int d = 0; d < 3; ++d)
            if ((rc = c->dalloc(&R.f[d], m * c->prec)) || (rc = c->dalloc(&R.u[d], m * c->prec)))
                return init_fail(c, rc, "");
    }
    {
        size_t m = (size_t)c->cap;
        if ((rc = c->dalloc((void **)&c->W.key, 4 * m)) || (rc = c->dalloc((void **)&c->W.rank, 4 * m)) ||
            (rc = c->dalloc((void **)&c->W.table, 4 * m)))
            return init_fail(c, rc, "");
    }
    c->Q.ncls = 64;
    if ((rc = c->dalloc((void **)&c->Q.cls_cnt, sizeof(int) * kSubQueues * c->Q.ncls)) ||
        (rc = c->dalloc((void **)&c->Q.cursor, sizeof(int) * kSubQueues * c->Q.ncls)) ||
        (rc = c->dalloc((void **)&c->Q.queue_bounds, sizeof(int) * (kSubQueues + 1))) ||
        (rc = c->dalloc((void **)&c->Q.queue_head, sizeof(int) * kSubQueues)))
        return init_fail(c, rc, "");
    if ((rc = c->dalloc((void **)&c->d_cycles, 8 * (size_t)n_boxes)) ||
        (rc = c->dalloc((void **)&c->d_rtc, 8 * (size_t)n_boxes)) ||
        (rc = c->dalloc((void **)&c->d_slow, sizeof(unsigned))) ||
        (rc = c->dalloc((void **)&c->d_slown, 2 * sizeof(unsigned))) ||
        (rc = c->dalloc((void **)&c->d_jdirty[0], sizeof(int) * (size_t)c->n[2])) ||
        (rc = c->dalloc((void **)&c->d_jdirty[1], sizeof(int) * (size_t)c->n[2])) ||
        (rc = c->dalloc((void **)&c->d_ylists, sizeof(int) * (4 * (size_t)c->n[2] + 4))) ||
        (rc = c->dalloc((void **)&c->d_counts, 8 * (size_t)n_boxes * n_species)))
        return init_fail(c, rc, "");
    // box geometry
    std::vector<int> lo(3 * n_boxes), hi(3 * n_boxes), b6(6 * n_boxes);
    for (int b = 0; b < n_boxes; ++b)
        for (int d = 0; d < 3; ++d) {
            lo[3 * b + d] = boxes[b].lo[d];
            hi[3 * b + d] = boxes[b].hi[d];
            b6[6 * b + d] = boxes[b].lo[d];
            b6[6 * b + 3 + d] = boxes[b].hi[d];
        }
    if ((rc = c->dalloc((void **)&c->d_box_lo, sizeof(int) * 3 * n_boxes)) ||
        (rc = c->dalloc((void **)&c->d_box_hi, sizeof(int) * 3 * n_boxes)) ||
        (rc = c->dalloc((void **)&c->d_boxes6, sizeof(int) * 6 * n_boxes)) ||
        (rc = c->dalloc((void **)&c->d_coarse_box, sizeof(int) * coarse.size())))
        return init_fail(c, rc, "");
    auto h2d = [&](void *d, const void *h, size_t bytes) { return hipMemcpy(d, h, bytes, hipMemcpyHostToDevice); };
    if (h2d(c->d_box_lo, lo.data(), sizeof(int) * lo.size()) || h2d(c->d_box_hi, hi.data(), sizeof(int) * hi.size()) ||
        h2d(c->d_boxes6, b6.data(), sizeof(int) * b6.size()) ||
        h2d(c->d_coarse_box, coarse.data(), sizeof(int) * coarse.size()))
        return init_fail(c, PIC_EDEVICE, "hipMemcpy of box tables failed");
    {
        BoxMap bm;
        bm.boxes6 = c->d_boxes6;
        bm.coarse_box = c->d_coarse_box;
        for (int d = 0; d < 3; ++d) {
            bm.g[d] = c->g[d];
            bm.cg[d] = c->cg[d];
        }
        if ((rc = c->dalloc((void **)&c->d_bmap, sizeof(BoxMap)))) return init_fail(c, rc, "");
        if (h2d(c->d_bmap, &bm, sizeof(BoxMap))) return init_fail(c, PIC_EDEVICE, "hipMemcpy of the box map failed");
    }
    if ((rc = c->build_tiles())) return init_fail(c, rc, "");

    // fields: E = J = 0, B = b_ext (stored as B - b_ext: the uniform part is
    // added at the gather, so single precision keeps the self-field's digits)
    for (int k = 0; k < 3; ++k) {
        if (launch_fill_f(c->prec, c->Eb[0][k], 0.0, N, c->st) || launch_fill_f(c->prec, c->Bb[0][k], 0.0, N, c->st) ||
            launch_fill_f(c->prec, c->Eb[1][k], 0.0, N, c->st) || launch_fill_f(c->prec, c->Bb[1][k], 0.0, N, c->st) ||
            launch_fill_f(c->prec, c->Jb[0][k], 0.0, N, c->st) || launch_fill_f(c->prec, c->Jb[1][k], 0.0, N, c->st))
            return init_fail(c, PIC_EDEVICE, "field initialisation failed");
    }
    if (launch_fill_u64(c->d_cycles, n_boxes, c->st) || launch_fill_u64(c->d_rtc, n_boxes, c->st) ||
        launch_fill_u32((uint32_t *)c->d_slow, 1, c->st) || launch_fill_u32((uint32_t *)c->d_slown, 2, c->st) ||
        c->mark_j_dirty() ||
        launch_fill_u32((uint32_t *)c->Q.cls_cnt, (size_t)kSubQueues * c->Q.ncls, c->st))
        return init_fail(c, PIC_EDEVICE, "counter initialisation failed");

    // particles: on-device Philox loader, species after species
    int64_t base = 0;
    for (int s = 0; s < n_species; ++s) {
        const pic_species_desc &S = species[s];
        if (S.load_mode == 0 || c->sp[s].count == 0) continue;
        LoadArgs a{};
        a.mode = S.load_mode;
        a.ppc = S.ppc;
        for (int d = 0; d < 3; ++d) {
            a.rlo[d] = S.region_lo[d];
            a.rext[d] = S.region_hi[d] - S.region_lo[d];
            a.uth[d] = S.u_th[d];
            a.udrift[d] = S.u_drift[d];
        }
        a.density = S.density;
        a.n = c->sp[s].count;
        a.out_base = base;
        a.species = s;
        a.k0 = (uint32_t)(c->seed & 0xffffffffu);
        a.k1 = (uint32_t)((c->seed >> 32) & 0xffffffffu) ^ (uint32_t)s;
        a.nb = n_boxes;
        a.boxes6 = c->d_boxes6;
        int64_t *d_base = nullptr;
        int32_t *d_ppc = nullptr;
        if (S.load_mode == 2) {
            std::vector<int64_t> bb(n_boxes + 1, 0);
            for (int b = 0; b < n_boxes; ++b) bb[b + 1] = bb[b] + box_cells[b] * S.box_ppc[b];
            if ((rc = c->dalloc((void **)&d_base, 8 * bb.size())) || (rc = c->dalloc((void **)&d_ppc, 4 * n_boxes)))
                return init_fail(c, rc, "");
            if (h2d(d_base, bb.data(), 8 * bb.size()) || h2d(d_ppc, S.box_ppc, 4 * (size_t)n_boxes))
                return init_fail(c, PIC_EDEVICE, "hipMemcpy failed");
            a.box_base = d_base;
            a.box_ppc = d_ppc;
        }
        if (launch_load(c->prec, c->P[c->pcur], a, c->st) != hipSuccess)
            return init_fail(c, PIC_EDEVICE, "particle loader launch failed");
        base += c->sp[s].count;
    }
    // make the compiled kernel variant's LDS limit known before any capture
    {
        GpdLaunch L = c->gpd_args();
        if (launch_gpd(c->prec, c->order, L, c->st) != hipSuccess)
            return init_fail(c, PIC_EDEVICE, "kernel attribute setup failed");
    }
    if ((rc = c->sort_now())) return init_fail(c, rc, "");
    if (hipStreamSynchronize(c->st) != hipSuccess) return init_fail(c, PIC_EDEVICE, "initialisation failed on device");
    *out = c;
    return PIC_OK;
}

PIC_API void pic_finalize(pic_ctx *ctx) { delete ctx; }

#define CHECK_CTX(ctx)                          \
    do {                                        \
        if (!(ctx)) return PIC_EINVAL;          \
        if ((ctx)->sticky) return (ctx)->sticky; \
    } while (0)

PIC_API int pic_step(pic_ctx *ctx, int32_t n_steps) {
    CHECK_CTX(ctx);
    if (n_steps < 0) return ctx->fail(PIC_EINVAL, "n_steps < 0");
    return ctx->step(n_steps);
}

PIC_API int pic_sync(pic_ctx *ctx) {
    CHECK_CTX(ctx);
    hipError_t e = hipStreamSynchronize(ctx->st);
    return e == hipSuccess ? PIC_OK : ctx->hip_fail(e, "hipStreamSynchronize");
}

PIC_API int pic_set_launch_mode(pic_ctx *ctx, int32_t mode, int32_t use_graph) {
    CHECK_CTX(ctx);
    if (mode < PIC_LAUNCH_PER_BOX || mode > PIC_LAUNCH_PERSISTENT) return ctx->fail(PIC_EINVAL, "bad launch mode");
    ctx->mode = mode;
    ctx->use_graph = use_graph != 0;
    ctx->drop_graphs();
    return PIC_OK;
}

PIC_API int pic_get_tuning(pic_ctx *ctx, pic_tuning *out) {
    CHECK_CTX(ctx);
    if (!out) return ctx->fail(PIC_EINVAL, "null output");
    *out = ctx->tun;
    return PIC_OK;
}

PIC_API int pic_set_tuning(pic_ctx *ctx, const pic_tuning *t) {
    CHECK_CTX(ctx);
    if (!t) return ctx->fail(PIC_EINVAL, "null tuning");
    if (t->block != 256 && t->block != 384 && t->block != 512)
        return ctx->fail(PIC_EINVAL, "block must be 256, 384 or 512");
    if (t->chunk < 64 || t->sort_interval < 1 || t->blocks_per_cu < 1 || t->blocks_per_cu > 16)
        return ctx->fail(PIC_EINVAL, "chunk >= 64, sort_interval >= 1, 1 <= blocks_per_cu <= 16");
    if (t->run_sum != 0 && t->run_sum != 1) return ctx->fail(PIC_EINVAL, "run_sum must be 0 or 1");
    if (t->field_overlap != 0 && t->field_overlap != 1)
        return ctx->fail(PIC_EINVAL, "field_overlap must be 0 or 1");
    if (!gpd_supported(t->tile, t->halo)) return ctx->fail(PIC_EUNSUPPORTED, "tile shape not compiled");
    if (gpd_lds_bytes(ctx->prec, ctx->order, t->tile, t->halo, t->block) > kLdsPerCu)
        return ctx->fail(PIC_EUNSUPPORTED, "tile needs more LDS than a CU has");
    for (int b = 0; b < ctx->nb; ++b)
        for (int d = 0; d < 3; ++d)
            if ((ctx->boxes[b].hi[d] - ctx->boxes[b].lo[d]) % t->tile[d])
                return ctx->fail(PIC_EUNSUPPORTED, "tile edge does not divide a box edge");
    hipError_t e = hipStreamSynchronize(ctx->st);
    if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamSynchronize");
    bool retile = std::memcmp(t->tile, ctx->tun.tile, sizeof(int) * 3) != 0 || t->chunk != ctx->tun.chunk;
    ctx->tun = *t;
    ctx->drop_graphs();
    int rc;
    if (retile && (rc = ctx->build_tiles())) return rc;
    {
        GpdLaunch L = ctx->gpd_args();
        e = launch_gpd(ctx->prec, ctx->order, L, ctx->st);
        if (e != hipSuccess) return ctx->hip_fail(e, "kernel attribute setup");
    }
    return ctx->sort_now();
}

// Copy of the mutable state (particles, fields, cost counters) used by the
// autotuner so that its trial steps leave the simulation untouched.
struct StateBackup {
    std::vector<void *> bufs;
    ~StateBackup() {
        for (void *p : bufs) (void)hipFree(p);
    }
};

static int copy_state(pic_ctx *c, StateBackup &bk, bool save) {
    size_t m = (size_t)c->np, N = (size_t)c->n[0] * c->n[1] * c->n[2], fb = N * c->prec;
    const ParticlesRaw &R = c->P[c->pcur];
    struct Item {
        void *dev;
        size_t bytes;
    };
    std::vector<Item> items = {{R.cell, 4 * m}, {R.id, 8 * m}, {R.sp, m}, {R.w, m * c->prec}};
    for (int d = 0; d < 3; ++d) {
        items.push_back({R.f[d], m * c->prec});
        items.push_back({R.u[d], m * c->prec});
        items.push_back({c->Eb[c->jcur][d], fb});
        items.push_back({c->Bb[c->jcur][d], fb});
        items.push_back({c->Jb[0][d], fb});
        items.push_back({c->Jb[1][d], fb});
    }
    items.push_back({c->d_cycles, 8 * (size_t)c->nb});
    items.push_back({c->d_rtc, 8 * (size_t)c->nb});
    if (save) {
        for (auto &it : items) {
            void *p = nullptr;
            hipError_t e = hipMalloc(&p, std::max<size_t>(16, it.bytes));
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return c->fail(PIC_ENOMEM, "autotune: no memory for a state copy");
            }
            bk.bufs.push_back(p);
        }
    }
    if (!save) {
        c->xvalid = false;
        if (c->mark_j_dirty()) return c->fail(PIC_EDEVICE, "J plane flags");
    }
    for (size_t i = 0; i < items.size(); ++i) {
        if (!items[i].bytes) continue;
        hipError_t e = save ? hipMemcpyAsync(bk.bufs[i], items[i].dev, items[i].bytes, hipMemcpyDeviceToDevice, c->st)
                            : hipMemcpyAsync(items[i].dev, bk.bufs[i], items[i].bytes, hipMemcpyDeviceToDevice, c->st);
        if (e != hipSuccess) return c->hip_fail(e, "autotune state copy");
    }
    hipError_t e = hipStreamSynchronize(c->st);
    return e == hipSuccess ? PIC_OK : c->hip_fail(e, "autotune sync");
}

static std::string tune_key(const pic_ctx *c) {
    // box-size mix, particle-count bucket, order, precision, launch mode
    std::map<std::string, int> sizes;
    for (const pic_box &b : c->boxes)
        sizes[std::to_string(b.hi[0] - b.lo[0]) + "x" + std::to_string(b.hi[1] - b.lo[1]) + "x" +
              std::to_string(b.hi[2] - b.lo[2])] += 1;
    std::string k;
    for (auto &kv : sizes) k += kv.first + ":" + std::to_string(kv.second) + ",";
    int bucket = 0;
    for (int64_t v = c->np; v > 1; v >>= 1) ++bucket;
    return k + "|np2^" + std::to_string(bucket) + "|m" + std::to_string(c->order) + "|p" + std::to_string(c->prec) +
           "|mode" + std::to_string(c->mode) + "|nsp" + std::to_string(c->nsp);
}

PIC_API int pic_autotune(pic_ctx *ctx, int32_t steps, pic_tuning *best, double *ms_per_step) {
    CHECK_CTX(ctx);
    if (steps < 1) return ctx->fail(PIC_EINVAL, "steps must be >= 1");
    std::string key = tune_key(ctx);
    auto hit = g_tune_cache.find(key);
    if (hit != g_tune_cache.end()) {
        int rc = pic_set_tuning(ctx, &hit->second);
        if (rc) return rc;
        if (best) *best = hit->second;
        if (ms_per_step) *ms_per_step = -1.0;
        return PIC_OK;
    }
    // candidates: every compiled tile that fits, three block sizes; then the
    // other particle order, and chunk and residency for the persistent queue,
    // around the best of those
    std::vector<pic_tuning> cand;
    const int tiles[4][3] = {{8, 4, 4}, {4, 4, 4}, {8, 8, 4}, {8, 8, 8}};
    pic_tuning base = ctx->tun;
    for (auto &t : tiles) {
        bool ok = true;
        for (int b = 0; b < ctx->nb && ok; ++b)
            for (int d = 0; d < 3; ++d)
                if ((ctx->boxes[b].hi[d] - ctx->boxes[b].lo[d]) % t[d]) ok = false;
        if (!ok) continue;
        for (int blk : {256, 384, 512}) {
            if (gpd_lds_bytes(ctx->prec, ctx->order, t, 1, blk) > kLdsPerCu) continue;
            pic_tuning c = base;
            std::memcpy(c.tile, t, sizeof(int) * 3);
            c.block = blk;
            c.blocks_per_cu = resident_blocks(ctx->prec, ctx->order, t, blk);
            cand.push_back(c);
        }
    }
    if (cand.empty()) return ctx->fail(PIC_EUNSUPPORTED, "no compiled tile fits these boxes");
    StateBackup bk;
    int rc = copy_state(ctx, bk, true);
    if (rc) return rc;
    int saved_jcur = ctx->jcur;
    int64_t saved_step = ctx->step_no;
    bool saved_graph = ctx->use_graph, saved_timing = ctx->timing;
    ctx->use_graph = false;
    ctx->timing = false;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return ctx->fail(PIC_EDEVICE, "autotune: hipEventCreate");
    // the field buffers to restore are those of the saved step's parity
    auto trial = [&](const pic_tuning &t, double &ms) -> int {
        ctx->jcur = saved_jcur;
        int r = copy_state(ctx, bk, false);
        if (r) return r;
        r = pic_set_tuning(ctx, &t);
        if (r) return r;
        if ((r = ctx->step(1))) return r;
        if (hipEventRecord(a, ctx->st) != hipSuccess) return ctx->fail(PIC_EDEVICE, "event");
        if ((r = ctx->step(steps))) return r;
        if (hipEventRecord(b, ctx->st) != hipSuccess || hipEventSynchronize(b) != hipSuccess)
            return ctx->fail(PIC_EDEVICE, "event");
        float f = 0.f;
        (void)hipEventElapsedTime(&f, a, b);
        ms = f / steps;
        return PIC_OK;
    };
    pic_tuning win = cand[0];
    double win_ms = 1e30;
    for (auto &t : cand) {
        double ms;
        if ((rc = trial(t, ms))) break;
        if (ms < win_ms) {
            win_ms = ms;
            win = t;
        }
    }
    if (!rc) {
        pic_tuning t = win;
        t.run_sum = 1 - win.run_sum;
        double ms;
        rc = trial(t, ms);
        if (!rc && ms < win_ms) {
            win_ms = ms;
            win = t;
        }
    }
    if (!rc && ctx->mode == PIC_LAUNCH_PERSISTENT) {
        const int fit = resident_blocks(ctx->prec, ctx->order, win.tile, win.block);
        for (int chunk : {1024, 2048, 4096, 8192}) {
            for (int bpc : {fit - 1, fit, fit + 1}) {
                if (bpc < 1 || (chunk == win.chunk && bpc == win.blocks_per_cu)) continue;
                pic_tuning t = win;
                t.chunk = chunk;
                t.blocks_per_cu = bpc;
                double ms;
                if ((rc = trial(t, ms))) break;
                if (ms < win_ms) {
                    win_ms = ms;
                    win = t;
                }
            }
            if (rc) break;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    ctx->jcur = saved_jcur;
    if ((rc = copy_state(ctx, bk, false))) return rc;
    if ((rc = pic_set_tuning(ctx, &win))) return rc;
    ctx->step_no = saved_step;
    ctx->use_graph = saved_graph;
    ctx->timing = saved_timing;
    ctx->drop_graphs();
    g_tune_cache[key] = win;
    if (best) *best = win;
    if (ms_per_step) *ms_per_step = win_ms;
    return PIC_OK;
}

PIC_API int pic_reset_costs(pic_ctx *ctx) {
    CHECK_CTX(ctx);
    if (launch_fill_u64(ctx->d_cycles, ctx->nb, ctx->st) || launch_fill_u64(ctx->d_rtc, ctx->nb, ctx->st))
        return ctx->fail(PIC_EDEVICE, "reset failed");
    return PIC_OK;
}

PIC_API int pic_box_counts(pic_ctx *ctx, int64_t *counts) {
    CHECK_CTX(ctx);
    if (!counts) return ctx->fail(PIC_EINVAL, "null counts");
    size_t m = (size_t)ctx->nb * ctx->nsp;
    hipError_t e;
    if ((e = launch_fill_u64(ctx->d_counts, m, ctx->st)) != hipSuccess) return ctx->hip_fail(e, "fill");
    if ((e = launch_box_counts(ctx->prec, ctx->P[ctx->pcur], (int)ctx->np, ctx->geom(), ctx->d_counts, ctx->st)) !=
        hipSuccess)
        return ctx->hip_fail(e, "box counts");
    if ((e = hipMemcpyAsync(counts, ctx->d_counts, 8 * m, hipMemcpyDeviceToHost, ctx->st)) != hipSuccess)
        return ctx->hip_fail(e, "copy counts");
    if ((e = hipStreamSynchronize(ctx->st)) != hipSuccess) return ctx->hip_fail(e, "sync");
    return PIC_OK;
}

PIC_API int pic_box_costs(pic_ctx *ctx, int32_t strategy, double *costs, int32_t *used_strategy) {
    CHECK_CTX(ctx);
    if (!costs) return ctx->fail(PIC_EINVAL, "null costs");
    int nb = ctx->nb;
    if (strategy == PIC_COST_DEVICE_TIMER || strategy == PIC_COST_DEVICE_RTC) {
        std::vector<unsigned long long> v(nb);
        const unsigned long long *src = strategy == PIC_COST_DEVICE_TIMER ? ctx->d_cycles : ctx->d_rtc;
        hipError_t e = hipMemcpyAsync(v.data(), src, 8 * (size_t)nb, hipMemcpyDeviceToHost, ctx->st);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
        if (e != hipSuccess) return ctx->hip_fail(e, "copy costs");
        for (int b = 0; b < nb; ++b) costs[b] = (double)v[b];
        if (strategy == PIC_COST_DEVICE_TIMER) ctx->last_timer.assign(costs, costs + nb);
        if (used_strategy) *used_strategy = strategy;
        return PIC_OK;
    }
    if (strategy == PIC_COST_HEURISTIC || strategy == PIC_COST_LEARNED) {
        if (strategy == PIC_COST_LEARNED) {
            int used = PIC_COST_HEURISTIC;
            int rc = ctx->learned_costs(costs, &used);
            if (rc) return rc;
            if (used == PIC_COST_LEARNED) {
                if (used_strategy) *used_strategy = used;
                return PIC_OK;
            }
        }
        std::vector<int64_t> cnt((size_t)nb * ctx->nsp);
        int rc = pic_box_counts(ctx, cnt.data());
        if (rc) return rc;
        std::vector<int64_t> tot(nb, 0), cells(nb);
        for (int b = 0; b < nb; ++b) {
            for (int s = 0; s < ctx->nsp; ++s) tot[b] += cnt[(size_t)b * ctx->nsp + s];
            const pic_box &B = ctx->boxes[b];
            cells[b] = (int64_t)(B.hi[0] - B.lo[0]) * (B.hi[1] - B.lo[1]) * (B.hi[2] - B.lo[2]);
        }
        pb_heuristic_costs(nb, tot.data(), cells.data(), ctx->wp, ctx->wc, costs);
        if (used_strategy) *used_strategy = PIC_COST_HEURISTIC;
        return PIC_OK;
    }
    return ctx->fail(PIC_EINVAL, "unknown cost strategy");
}

PIC_API int pic_get_particles(pic_ctx *ctx, int32_t species, double *x3, double *u3, double *w, int64_t *id,
                              int64_t *n_inout) {
    CHECK_CTX(ctx);
    if (!n_inout || species < 0 || species >= ctx->nsp) return ctx->fail(PIC_EINVAL, "bad species or null count");
    std::vector<uint32_t> cell;
    std::vector<double> f[3], u[3], wv;
    std::vector<int64_t> idv;
    std::vector<uint8_t> spv;
    int rc = ctx->download(cell, f, u, wv, idv, spv);
    if (rc) return rc;
    int64_t cap_out = *n_inout, k = 0;
    for (size_t i = 0; i < cell.size(); ++i) {
        if (spv[i] != species) continue;
        if (k < cap_out) {
            int c[3];
            unpack_cell(cell[i], c[0], c[1], c[2]);
            for (int d = 0; d < 3; ++d) {
                if (x3) x3[3 * k + d] = (double)c[d] + f[d][i];
                if (u3) u3[3 * k + d] = u[d][i];
            }
            if (w) w[k] = wv[i];
            if (id) id[k] = idv[i];
        }
        ++k;
    }
    *n_inout = k;
    return k > cap_out ? PIC_ECAPACITY : PIC_OK;
}

PIC_API int pic_get_particles_by_id(pic_ctx *ctx, int32_t species, const int64_t *ids, int64_t n, double *x3,
                                    double *u3, int32_t *found) {
    CHECK_CTX(ctx);
    if (species < 0 || species >= ctx->nsp || n < 0 || n > (int64_t)1 << 24 ||
        (n > 0 && (!ids || !x3 || !u3 || !found)))
        return ctx->fail(PIC_EINVAL, "bad species, count (0..2^24) or null arrays");
    if (n == 0) return PIC_OK;
    std::vector<int64_t> order(n), q(n);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return ids[a] < ids[b]; });
    for (int64_t k = 0; k < n; ++k) q[k] = ids[order[k]];
    for (int64_t k = 1; k < n; ++k)
        if (q[k] == q[k - 1]) return ctx->fail(PIC_EINVAL, "repeated id");
    const size_t P = (size_t)ctx->prec;
    void *dq = nullptr, *dcell = nullptr, *df = nullptr, *du = nullptr, *dfound = nullptr;
    auto release = [&]() {
        for (void *b : {dq, dcell, df, du, dfound})
            if (b) (void)hipFree(b);
    };
    hipError_t e = hipMalloc(&dq, 8 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&dcell, 4 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&df, 3 * P * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&du, 3 * P * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&dfound, 4 * (size_t)n);
    if (e != hipSuccess) {
        release();
        (void)hipGetLastError();
        return ctx->fail(PIC_ENOMEM, "no device memory for the id lookup");
    }
    e = hipMemcpyAsync(dq, q.data(), 8 * (size_t)n, hipMemcpyHostToDevice, ctx->st);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t *)dfound, (size_t)n, ctx->st);
    if (e == hipSuccess)
        e = launch_find_ids(ctx->prec, ctx->P[ctx->pcur], (int)ctx->np, species, (const int64_t *)dq, (int)n,
                            (uint32_t *)dcell, df, du, (int *)dfound, ctx->st);
    std::vector<uint32_t> cell(n);
    std::vector<int32_t> fnd(n);
    std::vector<unsigned char> fb(3 * P * (size_t)n), ub(3 * P * (size_t)n);
    if (e == hipSuccess) e = hipMemcpyAsync(cell.data(), dcell, 4 * (size_t)n, hipMemcpyDeviceToHost, ctx->st);
    if (e == hipSuccess) e = hipMemcpyAsync(fnd.data(), dfound, 4 * (size_t)n, hipMemcpyDeviceToHost, ctx->st);
    if (e == hipSuccess) e = hipMemcpyAsync(fb.data(), df, fb.size(), hipMemcpyDeviceToHost, ctx->st);
    if (e == hipSuccess) e = hipMemcpyAsync(ub.data(), du, ub.size(), hipMemcpyDeviceToHost, ctx->st);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
    release();
    if (e != hipSuccess) return ctx->hip_fail(e, "id lookup");
    auto val = [&](const std::vector<unsigned char> &b, size_t i) -> double {
        if (P == 8) return ((const double *)b.data())[i];
        return (double)((const float *)b.data())[i];
    };
    for (int64_t k = 0; k < n; ++k) {
        const int64_t o = order[k];
        found[o] = fnd[k];
        int c[3];
        unpack_cell(cell[k], c[0], c[1], c[2]);
        for (int d = 0; d < 3; ++d) {
            x3[3 * o + d] = fnd[k] ? (double)c[d] + val(fb, 3 * (size_t)k + d) : 0.0;
            u3[3 * o + d] = fnd[k] ? val(ub, 3 * (size_t)k + d) : 0.0;
        }
    }
    return PIC_OK;
}

PIC_API int pic_set_particles(pic_ctx *ctx, int32_t species, const double *x3, const double *u3, const double *w,
                              const int64_t *id, int64_t n) {
    CHECK_CTX(ctx);
    if (species < 0 || species >= ctx->nsp || n < 0 || (n > 0 && (!x3 || !u3 || !w)))
        return ctx->fail(PIC_EINVAL, "bad species, count or null arrays");
    if (n > ctx->sp[species].cap) return ctx->fail(PIC_ECAPACITY, "more particles than the species' capacity");
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d)
            if (!(x3[3 * i + d] >= 0.0 && x3[3 * i + d] < (double)ctx->n[d]))
                return ctx->fail(PIC_EINVAL, "position outside [0, n)");
    std::vector<uint32_t> cell;
    std::vector<double> f[3], u[3], wv;
    std::vector<int64_t> idv;
    std::vector<uint8_t> spv;
    int rc = ctx->download(cell, f, u, wv, idv, spv);
    if (rc) return rc;
    // keep other species, append the new ones
    size_t k = 0;
    for (size_t i = 0; i < cell.size(); ++i) {
        if (spv[i] == species) continue;
        cell[k] = cell[i];
        for (int d = 0; d < 3; ++d) {
            f[d][k] = f[d][i];
            u[d][k] = u[d][i];
        }
        wv[k] = wv[i];
        idv[k] = idv[i];
        spv[k] = spv[i];
        ++k;
    }
    size_t m = k + (size_t)n;
    cell.resize(m);
    idv.resize(m);
    spv.resize(m);
    wv.resize(m);
    for (int d = 0; d < 3; ++d) {
        f[d].resize(m);
        u[d].resize(m);
    }
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        for (int d = 0; d < 3; ++d) {
            double x = x3[3 * i + d];
            double fl = std::floor(x);
            double off = x - fl;
            int ci = (int)fl;
            if (ctx->prec == PIC_FP32 && (double)(float)off >= 1.0) {
                off = 0.0;
                ci += 1;
            }
            if (ci >= ctx->n[d]) ci -= ctx->n[d];
            c[d] = ci;
            f[d][k + i] = off;
            u[d][k + i] = u3[3 * i + d];
        }
        cell[k + i] = pack_cell(c[0], c[1], c[2]);
        wv[k + i] = w[i];
        idv[k + i] = id ? id[i] : i;
        spv[k + i] = (uint8_t)species;
    }
    ctx->sp[species].count = n;
    return ctx->upload(cell, f, u, wv, idv, spv);
}

PIC_API int pic_get_field(pic_ctx *ctx, int32_t comp, double *out) {
    CHECK_CTX(ctx);
    if (!out || comp < 0 || comp > 8) return ctx->fail(PIC_EINVAL, "bad component or null output");
    const void *src = comp < 3   ? ctx->Eb[ctx->jcur][comp]
                      : comp < 6 ? ctx->Bb[ctx->jcur][comp - 3]
                                 : ctx->Jb[1 - ctx->jcur][comp - 6];
    size_t N = (size_t)ctx->n[0] * ctx->n[1] * ctx->n[2];
    hipError_t e = hipStreamSynchronize(ctx->st);
    if (e != hipSuccess) return ctx->hip_fail(e, "sync");
    if (ctx->prec == 8) {
        e = hipMemcpy(out, src, 8 * N, hipMemcpyDeviceToHost);
    } else {
        std::vector<float> t(N);
        e = hipMemcpy(t.data(), src, 4 * N, hipMemcpyDeviceToHost);
        for (size_t i = 0; i < N; ++i) out[i] = t[i];
    }
    if (comp >= 3 && comp < 6 && ctx->bext[comp - 3] != 0.0)
        for (size_t i = 0; i < N; ++i) out[i] += ctx->bext[comp - 3];
    return e == hipSuccess ? PIC_OK : ctx->hip_fail(e, "copy field");
}

PIC_API int pic_set_field(pic_ctx *ctx, int32_t comp, const double *in) {
    CHECK_CTX(ctx);
    if (!in || comp < 0 || comp > 8) return ctx->fail(PIC_EINVAL, "bad component or null input");
    void *dst = comp < 3   ? ctx->Eb[ctx->jcur][comp]
                : comp < 6 ? ctx->Bb[ctx->jcur][comp - 3]
                           : ctx->Jb[1 - ctx->jcur][comp - 6];
    size_t N = (size_t)ctx->n[0] * ctx->n[1] * ctx->n[2];
    hipError_t e = hipStreamSynchronize(ctx->st);
    if (e != hipSuccess) return ctx->hip_fail(e, "sync");
    double off = comp >= 3 && comp < 6 ? ctx->bext[comp - 3] : 0.0;
    if (comp < 6) ctx->xvalid = false;  // the half-step B follows E and B
    else if (ctx->mark_j_dirty()) return ctx->fail(PIC_EDEVICE, "J plane flags");
    if (ctx->prec == 8) {
        std::vector<double> t(in, in + N);
        for (size_t i = 0; i < N; ++i) t[i] -= off;
        e = hipMemcpy(dst, t.data(), 8 * N, hipMemcpyHostToDevice);
    } else {
        std::vector<float> t(N);
        for (size_t i = 0; i < N; ++i) t[i] = (float)(in[i] - off);
        e = hipMemcpy(dst, t.data(), 4 * N, hipMemcpyHostToDevice);
    }
    return e == hipSuccess ? PIC_OK : ctx->hip_fail(e, "copy field");
}

PIC_API int pic_set_cost_timer(pic_ctx *ctx, int32_t enable) {
    CHECK_CTX(ctx);
    bool on = enable != 0;
    if (on != ctx->cost_timer) {
        hipError_t e = hipStreamSynchronize(ctx->st);
        if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamSynchronize");
        ctx->cost_timer = on;
        ctx->drop_graphs();
    }
    return PIC_OK;
}

PIC_API int pic_set_staging(pic_ctx *ctx, int32_t enable) {
    CHECK_CTX(ctx);
    bool on = enable != 0;
    if (on != ctx->staged) {
        hipError_t e = hipStreamSynchronize(ctx->st);
        if (e != hipSuccess) return ctx->hip_fail(e, "hipStreamSynchronize");
        ctx->staged = on;
        ctx->drop_graphs();
    }
    return PIC_OK;
}

PIC_API int pic_kernel_timing(pic_ctx *ctx, int32_t enable) {
    CHECK_CTX(ctx);
    ctx->timing = enable != 0;
    return PIC_OK;
}

PIC_API int pic_kernel_times(pic_ctx *ctx, double *ms, int64_t *launches) {
    CHECK_CTX(ctx);
    hipError_t e = hipStreamSynchronize(ctx->st);
    if (e != hipSuccess) return ctx->hip_fail(e, "sync");
    for (int k = 0; k < 4; ++k) {
        double tot = 0.0;
        for (auto &p : ctx->events[k]) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, p.first, p.second) == hipSuccess) tot += t;
        }
        if (ms) ms[k] = tot;
        if (launches) launches[k] = (int64_t)ctx->events[k].size();
    }
    return PIC_OK;
}

PIC_API int pic_slow_path_count(pic_ctx *ctx, int64_t *count) {
    CHECK_CTX(ctx);
    unsigned v = 0;
    hipError_t e = hipMemcpyAsync(&v, ctx->d_slow, sizeof(unsigned), hipMemcpyDeviceToHost, ctx->st);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
    if (e != hipSuccess) return ctx->hip_fail(e, "copy slow count");
    if (count) *count = v;
    if (launch_fill_u32((uint32_t *)ctx->d_slow, 1, ctx->st) != hipSuccess) return ctx->fail(PIC_EDEVICE, "reset");
    return PIC_OK;
}

PIC_API int pic_box_features(pic_ctx *ctx, float *feat) {
    CHECK_CTX(ctx);
    if (!feat) return ctx->fail(PIC_EINVAL, "null features");
    int rc = ctx->features_device();
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(feat, ctx->d_feat, sizeof(float) * 16 * ctx->nb, hipMemcpyDeviceToHost, ctx->st);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
    return e == hipSuccess ? PIC_OK : ctx->hip_fail(e, "copy features");
}

}  // extern "C"

// Computes the per-box features into d_feat (device).
int pic_ctx::features_device() {
    size_t N = (size_t)n[0] * n[1] * n[2];
    int rc;
    if (!FS.cellcount) {
        if ((rc = dalloc((void **)&FS.cellcount, 4 * N)) || (rc = dalloc((void **)&FS.spcnt, 16 * (size_t)nb)) ||
            (rc = dalloc((void **)&FS.edge, 8 * (size_t)nb)) || (rc = dalloc((void **)&FS.usum, 8 * (size_t)nb)) ||
            (rc = dalloc((void **)&d_feat, 64 * (size_t)nb)))
            return rc;
    }
    HIPC(launch_fill_u32(FS.cellcount, N, st));
    HIPC(launch_fill_u64(FS.spcnt, 2 * (size_t)nb, st));
    HIPC(launch_fill_u64(FS.edge, nb, st));
    HIPC(launch_fill_f64(FS.usum, nb, st));
    HIPC(launch_features(prec, P[pcur], (int)np, geom(), nb, d_box_hi, FS, d_feat, st));
    return PIC_OK;
}
