// Host side of the gather-push-deposit kernels: the compiled tile shapes,
// their LDS footprint and the dispatch to the kernel groups (one object per
// precision and shape order, built from gpd_inst.hip), and the global-path
// kernel.
#include "kernels.hpp"

#include <hip/hip_runtime.h>

namespace pb {

// Defined in gpd_kernel.hpp and instantiated once per (precision, order).
template <typename real, int M>
hipError_t gpd_tile(const GpdLaunch &L, hipStream_t st);
template <typename real, int M>
hipError_t gpd_global(const GpdLaunch &L, int n, unsigned grid, hipStream_t st);

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

hipError_t launch_gpd_global(int prec, int order, const GpdLaunch &L, int n, unsigned grid, hipStream_t st) {
    if (prec == 8) {
        if (order == 3) return gpd_global<double, 3>(L, n, grid, st);
        return order == 2 ? gpd_global<double, 2>(L, n, grid, st) : gpd_global<double, 1>(L, n, grid, st);
    }
    if (order == 3) return gpd_global<float, 3>(L, n, grid, st);
    return order == 2 ? gpd_global<float, 2>(L, n, grid, st) : gpd_global<float, 1>(L, n, grid, st);
}

}  // namespace pb
