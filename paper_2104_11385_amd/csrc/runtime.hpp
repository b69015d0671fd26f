// The library context (opaque pic_ctx of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "kernels.hpp"

// Heuristic per-box cost w_p * particles + w_c * cells, rounded as written
// (lb.cpp, compiled without floating-point contraction).
extern "C" void pb_heuristic_costs(int nb, const int64_t *particles, const int64_t *cells, double wp, double wc,
                                   double *costs);

namespace pb {
struct MlpState;
}

// Takes the device address of the no-allocation lookup's scratch array on
// device dev (current), once per device (noalloc.hip).
int pb_noalloc_setup(int dev, std::string &err);

struct pic_ctx {
    // problem
    int n[3] = {0, 0, 0};
    double dt = 0.0;
    int order = 1, prec = 4;
    uint64_t seed = 0;
    double wp = 0.75, wc = 0.25, bext[3] = {0, 0, 0};
    int nb = 0;
    std::vector<pic_box> boxes;
    int nsp = 0;
    struct Species {
        double q = 0, m = 1, density = 0;
        int mode = 0;
        int64_t count = 0, cap = 0;
        std::vector<int32_t> box_ppc;
    } sp[pb::kMaxSpecies];
    int64_t np = 0, cap = 0;

    // execution
    int dev = 0, n_cu = 256;
    hipStream_t st = nullptr;
    bool own_stream = false;
    // second stream for the field update of the z-planes out of the step's
    // deposit reach, forked from and joined back into st by events
    hipStream_t st2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    pic_tuning tun{};
    int mode = PIC_LAUNCH_PERSISTENT;
    bool use_graph = false;
    bool capturing = false;
    // captured steps, by [sort first][field buffer][particle buffer]
    hipGraphExec_t gexec[2][2][2] = {};
    int steps_since_sort = 0;
    int64_t step_no = 0;

    // geometry
    int g[3] = {1, 1, 1}, cg[3] = {1, 1, 1};
    int ntiles = 0;
    std::vector<int> h_box_tile_off;
    int *d_coarse_box = nullptr, *d_box_lo = nullptr, *d_box_hi = nullptr, *d_boxes6 = nullptr;
    int *d_box_nt = nullptr, *d_box_tile_off = nullptr;
    pb::TileDesc *d_tiles = nullptr;
    pb::BoxMap *d_bmap = nullptr;

    // state
    pb::ParticlesRaw P[2];
    int pcur = 0;
    // E, B and J are double-buffered; index jcur holds the current E and B
    // and is the J buffer the next step deposits into (all flip each step)
    void *Eb[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    void *Bb[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    void *Jb[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    // B half a step ahead of the current E: valid while no field was set
    // from outside since the last update
    void *Xb[3] = {nullptr, nullptr, nullptr};
    bool xvalid = false;
    int yee_half();
    pb::YeeBuffers yee_buffers() const;
    int mark_j_dirty();
    int jcur = 0;
    pb::SortScratch W{};
    pb::QueueScratch Q{};
    pb::FeatScratch FS{};
    float *d_feat = nullptr;

    // costs
    unsigned long long *d_cycles = nullptr, *d_rtc = nullptr, *d_counts = nullptr;
    unsigned *d_slow = nullptr;
    unsigned *d_slown = nullptr;  // [2] global-path list length and completion counter
    int *d_jdirty[2] = {nullptr, nullptr};  // per z-plane: J buffer b may be nonzero there
    int *d_ylists = nullptr;                 // [4 nz + 4] plane lists of the split field update
    std::vector<double> last_timer;      // last device-timer costs read
    std::vector<double> last_pred;       // learned prediction made for the current interval
    double mare = -1.0;                  // last mean relative error of the learned costs

    // timing
    bool timing = false;
    bool cost_timer = true;  // per-box clock counters in the gather-push-deposit kernel
    bool staged = true;      // tile windows staged in LDS (off: global-memory reference path)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events[4];
    std::pair<hipEvent_t, hipEvent_t> ev_pending{};
    int ev_kind = 0;

    // learned cost model
    pb::MlpState *mlp = nullptr;

    // bookkeeping
    std::vector<void *> allocs, tile_allocs;
    std::string err;
    int sticky = 0;

    ~pic_ctx();
    int fail(int code, const std::string &msg);
    int hip_fail(hipError_t e, const char *what);
    int dalloc(void **p, size_t bytes);
    pb::Geom geom() const;
    void drop_graphs();
    int build_tiles();
    void free_tile_buffers();
    int sort_now();
    pb::GpdLaunch gpd_args() const;
    int time_begin(int kind);
    int time_end();
    int enqueue_step();
    int step(int nsteps);
    int download(std::vector<uint32_t> &cell, std::vector<double> f[3], std::vector<double> u[3],
                 std::vector<double> &w, std::vector<int64_t> &id, std::vector<uint8_t> &spv);
    int upload(const std::vector<uint32_t> &cell, const std::vector<double> f[3], const std::vector<double> u[3],
               const std::vector<double> &w, const std::vector<int64_t> &id, const std::vector<uint8_t> &spv);
    int features_device();
    int learned_costs(double *costs, int *used);
    void mlp_release();
};
