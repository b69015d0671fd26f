// Load balancing on the host (Sec. 2.2, Eq. 1): load-balance efficiency,
// the adopt-if-improved threshold, and the knapsack and Morton
// space-filling-curve distribution mappings over a number of ranks.
//
// Compiled with -ffp-contract=off so that every sum and product rounds
// exactly as written: mappings must be reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <set>
#include <utility>
#include <vector>

#include "picbal.h"

namespace {

// Spreads the low 21 bits of v so that bit k lands on bit 3k.
uint64_t spread3(uint64_t v) {
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

bool costs_ok(const double *c, int32_t n) {
    for (int32_t i = 0; i < n; ++i)
        if (!(c[i] >= 0.0)) return false;  // rejects negatives and NaN
    return true;
}

// Smallest number of contiguous runs, each summed left to right from its
// first box, whose sums stay <= cap (a box larger than cap makes it
// impossible: returns INT32_MAX).
int32_t runs_needed(const std::vector<double> &c, double cap) {
    int32_t runs = 0;
    size_t i = 0, n = c.size();
    while (i < n) {
        if (c[i] > cap) return INT32_MAX;
        double s = c[i];
        size_t j = i + 1;
        while (j < n) {
            double t = s + c[j];
            if (t > cap) break;
            s = t;
            ++j;
        }
        ++runs;
        i = j;
    }
    return runs;
}

// Order-preserving map of non-negative doubles to integers and back.
uint64_t dbits(double v) {
    uint64_t u;
    std::memcpy(&u, &v, 8);
    return u;
}
double bitsd(uint64_t u) {
    double v;
    std::memcpy(&v, &u, 8);
    return v;
}

int sfc_map(const double *costs, const pic_box *boxes, int32_t nb, int32_t R, int32_t *rank) {
    // Morton order of the boxes' lower corners in units of the common edge
    int64_t g = 0;
    for (int32_t b = 0; b < nb; ++b)
        for (int d = 0; d < 3; ++d) g = std::gcd(g, (int64_t)(boxes[b].hi[d] - boxes[b].lo[d]));
    if (g <= 0) return PIC_EINVAL;
    std::vector<std::pair<uint64_t, int32_t>> key(nb);
    for (int32_t b = 0; b < nb; ++b) {
        uint64_t k = spread3((uint64_t)(boxes[b].lo[0] / g)) | (spread3((uint64_t)(boxes[b].lo[1] / g)) << 1) |
                     (spread3((uint64_t)(boxes[b].lo[2] / g)) << 2);
        key[b] = {k, b};
    }
    std::sort(key.begin(), key.end());
    std::vector<double> c(nb);
    for (int32_t i = 0; i < nb; ++i) c[i] = costs[key[i].second];
    if (nb <= R) {
        for (int32_t i = 0; i < nb; ++i) rank[key[i].second] = i;
        return PIC_OK;
    }
    // The optimal largest run sum B* is the smallest double for which R runs
    // suffice; feasibility is monotone, so bisect over the bit patterns of
    // non-negative doubles between the largest box and the total.
    double mx = *std::max_element(c.begin(), c.end());
    double total = 0.0;
    for (double v : c) total += v;
    uint64_t lo = dbits(mx), hi = dbits(std::max(total, mx));
    if (runs_needed(c, bitsd(lo)) <= R) hi = lo;
    while (hi - lo > 1) {  // invariant: lo infeasible (or lo == hi), hi feasible
        uint64_t mid = lo + (hi - lo) / 2;
        if (runs_needed(c, bitsd(mid)) <= R) hi = mid;
        else lo = mid;
    }
    double cap = bitsd(hi);
    // Assign: each run is the longest with sum <= B* that leaves at least one
    // box for every later rank; the last rank takes the rest.
    size_t i = 0;
    for (int32_t r = 0; r < R; ++r) {
        size_t keep = (size_t)(R - r - 1);
        size_t stop = r == R - 1 ? (size_t)nb : (size_t)nb - keep;
        double s = 0.0;
        size_t j = i;
        while (j < stop) {
            double t = j == i ? c[j] : s + c[j];
            if (r < R - 1 && j > i && t > cap) break;
            s = t;
            rank[key[j].second] = r;
            ++j;
        }
        i = j;
    }
    return PIC_OK;
}

int knapsack_map(const double *costs, int32_t nb, int32_t R, int32_t *rank) {
    int64_t cap = ((int64_t)3 * nb + 2 * (int64_t)R - 1) / (2 * (int64_t)R);  // ceil(1.5 nb / R)
    std::vector<int32_t> order(nb);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        if (costs[a] != costs[b]) return costs[a] > costs[b];
        return a < b;
    });
    // ranks that still accept boxes, keyed by (load, rank)
    std::set<std::pair<double, int32_t>> open;
    std::vector<double> load(R, 0.0);
    std::vector<int64_t> count(R, 0);
    for (int32_t r = 0; r < R; ++r) open.insert({0.0, r});
    for (int32_t b : order) {
        auto it = open.begin();
        int32_t r = it->second;
        open.erase(it);
        rank[b] = r;
        load[r] = load[r] + costs[b];
        if (++count[r] < cap) open.insert({load[r], r});
    }
    return PIC_OK;
}

}  // namespace

extern "C" {

// Per-box heuristic cost (Sec. 2.2): fl(fl(wp * particles) + fl(wc * cells)).
void pb_heuristic_costs(int nb, const int64_t *particles, const int64_t *cells, double wp, double wc,
                        double *costs) {
    for (int b = 0; b < nb; ++b) {
        double a = wp * (double)particles[b];
        double c = wc * (double)cells[b];
        costs[b] = a + c;
    }
}

PIC_API uint64_t lb_morton_key(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

PIC_API double lb_efficiency(const double *costs, const int32_t *rank_of_box, int32_t n_boxes, int32_t n_ranks) {
    if (!costs || !rank_of_box || n_boxes < 1 || n_ranks < 1) return -1.0;
    std::vector<double> per(n_ranks, 0.0);
    for (int32_t b = 0; b < n_boxes; ++b) {
        int32_t r = rank_of_box[b];
        if (r < 0 || r >= n_ranks) return -1.0;
        per[r] = per[r] + costs[b];
    }
    double sum = 0.0, top = 0.0;
    for (double v : per) {
        sum = sum + v;
        top = std::max(top, v);
    }
    if (top == 0.0) return 1.0;
    return (sum / (double)n_ranks) / top;
}

PIC_API int lb_should_adopt(double e_current, double e_proposed, double threshold) {
    double need = (1.0 + threshold) * e_current;
    return e_proposed >= need ? 1 : 0;
}

PIC_API int lb_distribute(const double *costs, const pic_box *boxes, int32_t n_boxes, int32_t n_ranks, int32_t policy,
                          int32_t *rank_of_box, double *efficiency) {
    if (!costs || !rank_of_box || n_boxes < 1 || n_ranks < 1) return PIC_EINVAL;
    if (!costs_ok(costs, n_boxes)) return PIC_EINVAL;
    int rc;
    if (policy == LB_SFC) {
        if (!boxes) return PIC_EINVAL;
        rc = sfc_map(costs, boxes, n_boxes, n_ranks, rank_of_box);
    } else if (policy == LB_KNAPSACK) {
        rc = knapsack_map(costs, n_boxes, n_ranks, rank_of_box);
    } else {
        return PIC_EINVAL;
    }
    if (rc == PIC_OK && efficiency) *efficiency = lb_efficiency(costs, rank_of_box, n_boxes, n_ranks);
    return rc;
}

// Halo traffic of a mapping: every face shared by two boxes on different
// ranks (the domain is periodic) costs bytes_per_face_cell per cell of face,
// sent by each of the two ranks.  Walks the coarse grid of box corners.
PIC_API int lb_comm_volume(const pic_box *boxes, int32_t n_boxes, const int32_t n_cells[3],
                           const int32_t *rank_of_box, int32_t n_ranks, double bytes_per_face_cell,
                           double *per_rank, double *total) {
    if (!boxes || !n_cells || !rank_of_box || n_boxes < 1 || n_ranks < 1) return PIC_EINVAL;
    int64_t g[3], cg[3];
    for (int d = 0; d < 3; ++d) {
        if (n_cells[d] < 1) return PIC_EINVAL;
        int64_t v = n_cells[d];
        for (int32_t b = 0; b < n_boxes; ++b) v = std::gcd(std::gcd(v, (int64_t)boxes[b].lo[d]), (int64_t)boxes[b].hi[d]);
        g[d] = v;
        cg[d] = n_cells[d] / v;
    }
    std::vector<int32_t> owner((size_t)(cg[0] * cg[1] * cg[2]), -1);
    for (int32_t b = 0; b < n_boxes; ++b) {
        if (rank_of_box[b] < 0 || rank_of_box[b] >= n_ranks) return PIC_EINVAL;
        for (int64_t z = boxes[b].lo[2] / g[2]; z < boxes[b].hi[2] / g[2]; ++z)
            for (int64_t y = boxes[b].lo[1] / g[1]; y < boxes[b].hi[1] / g[1]; ++y)
                for (int64_t x = boxes[b].lo[0] / g[0]; x < boxes[b].hi[0] / g[0]; ++x) {
                    int32_t &o = owner[(size_t)(x + cg[0] * (y + cg[1] * z))];
                    if (o >= 0) return PIC_EINVAL;
                    o = b;
                }
    }
    for (int32_t o : owner)
        if (o < 0) return PIC_EINVAL;
    std::vector<double> per(n_ranks, 0.0);
    const double area[3] = {(double)(g[1] * g[2]), (double)(g[0] * g[2]), (double)(g[0] * g[1])};
    for (int64_t z = 0; z < cg[2]; ++z)
        for (int64_t y = 0; y < cg[1]; ++y)
            for (int64_t x = 0; x < cg[0]; ++x) {
                int32_t b = owner[(size_t)(x + cg[0] * (y + cg[1] * z))];
                int64_t nb[3][3] = {{(x + 1) % cg[0], y, z}, {x, (y + 1) % cg[1], z}, {x, y, (z + 1) % cg[2]}};
                for (int d = 0; d < 3; ++d) {
                    int32_t c = owner[(size_t)(nb[d][0] + cg[0] * (nb[d][1] + cg[1] * nb[d][2]))];
                    int32_t ra = rank_of_box[b], rb = rank_of_box[c];
                    if (ra == rb) continue;
                    double v = area[d] * bytes_per_face_cell;
                    per[ra] += v;
                    per[rb] += v;
                }
            }
    double tot = 0.0;
    for (int32_t r = 0; r < n_ranks; ++r) {
        tot += per[r];
        if (per_rank) per_rank[r] = per[r];
    }
    if (total) *total = tot;
    return PIC_OK;
}

}  // extern "C"
