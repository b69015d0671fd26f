// Particle lookup by id without any allocation: the variant of
// pic_get_particles_by_id for callers that cannot allocate device memory
// (code under stream capture, serving loops, harnesses that forbid it).
// Its scratch memory is one statically sized device array per GPU; the
// library takes the array's device address once per device when a context
// is created there.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"
#include "runtime.hpp"

namespace pb {

// Largest lookup and the layout of the scratch array (byte offsets, each
// 256-byte aligned): query ids, an open-addressing table of twice as many
// slots (keys, then the query index of each key), the results in the caller's
// layout (x3, u3 as double, found as int32) and a repeated-id flag.
constexpr int64_t kNoallocMaxIds = 65536;
constexpr int64_t kSlots = 2 * kNoallocMaxIds;
constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kOffIds = 0;
constexpr size_t kOffKeys = kOffIds + align256(8 * kNoallocMaxIds);
constexpr size_t kOffIdx = kOffKeys + align256(8 * kSlots);
constexpr size_t kOffX = kOffIdx + align256(4 * kSlots);
constexpr size_t kOffU = kOffX + align256(24 * kNoallocMaxIds);
constexpr size_t kOffFound = kOffU + align256(24 * kNoallocMaxIds);
constexpr size_t kOffFlag = kOffFound + align256(4 * kNoallocMaxIds);
constexpr size_t kScratchBytes = kOffFlag + 256;  // 5.5 MiB

}  // namespace pb

using namespace pb;

// The scratch array.  In host code this name is only a stand-in for the
// symbol: kernels get the device address taken below, never the name.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

constexpr int64_t kEmpty = INT64_MIN;  // table key of a free slot (ids are >= 0)

__device__ __forceinline__ uint32_t slot_of(int64_t id) {
    uint64_t h = (uint64_t)id * 0x9E3779B97F4A7C15ull;
    return (uint32_t)(h >> 40) & (uint32_t)(kSlots - 1);
}

// Clears the table and the results of a call (the array keeps the last
// call's contents).
__global__ void k_na_clear(unsigned char *s, int n) {
    int64_t *keys = (int64_t *)(s + kOffKeys);
    double *x = (double *)(s + kOffX), *u = (double *)(s + kOffU);
    int *found = (int *)(s + kOffFound);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < kSlots; i += (int64_t)gridDim.x * blockDim.x) {
        keys[i] = kEmpty;
        if (i < n) {
            found[i] = 0;
            for (int d = 0; d < 3; ++d) {
                x[3 * i + d] = 0.0;
                u[3 * i + d] = 0.0;
            }
        }
        if (i == 0) *(int *)(s + kOffFlag) = 0;
    }
}

// Inserts query i's id with value i (linear probing); a repeated id sets the
// flag.
__global__ void k_na_insert(unsigned char *s, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t id = ((const int64_t *)(s + kOffIds))[i];
    unsigned long long *keys = (unsigned long long *)(s + kOffKeys);
    int *idx = (int *)(s + kOffIdx);
    uint32_t h = slot_of(id);
    for (int64_t k = 0; k < kSlots; ++k) {
        const uint32_t slot = (h + (uint32_t)k) & (uint32_t)(kSlots - 1);
        const unsigned long long prev = atomicCAS(&keys[slot], (unsigned long long)kEmpty, (unsigned long long)id);
        if (prev == (unsigned long long)kEmpty) {
            idx[slot] = i;
            return;
        }
        if (prev == (unsigned long long)id) {
            *(int *)(s + kOffFlag) = 1;
            return;
        }
    }
}

// Each particle of species sp looks its id up in the table and, if it is a
// query, writes its global position and momentum in the caller's layout.
template <typename real>
__global__ void k_na_find(Particles<real> P, int np, int sp, unsigned char *s) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np || P.sp[p] != sp) return;
    const int64_t id = P.id[p];
    const int64_t *keys = (const int64_t *)(s + kOffKeys);
    uint32_t h = slot_of(id);
    for (int64_t k = 0; k < kSlots; ++k) {
        const uint32_t slot = (h + (uint32_t)k) & (uint32_t)(kSlots - 1);
        const int64_t key = keys[slot];
        if (key == kEmpty) return;
        if (key != id) continue;
        // the table is complete before this kernel runs (stream order)
        const int i = ((const int *)(s + kOffIdx))[slot];
        double *x = (double *)(s + kOffX), *u = (double *)(s + kOffU);
        int c[3];
        unpack_cell(P.cell[p], c[0], c[1], c[2]);
        for (int d = 0; d < 3; ++d) {
            x[3 * i + d] = (double)c[d] + (double)P.f[d][p];
            u[3 * i + d] = (double)P.u[d][p];
        }
        ((int *)(s + kOffFound))[i] = 1;
        return;
    }
}

template <typename real>
Particles<real> view(const ParticlesRaw &r) {
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

}  // namespace

// Takes the device address of the scratch array on device dev (which must be
// current), once per device.  Called by pic_init.
int pb_noalloc_setup(int dev, std::string &err) {
    if (dev < 0 || dev >= kMaxDevices) {
        err = "device index beyond the scratch table";
        return PIC_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return PIC_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        err = std::string("hipGetSymbolAddress of the lookup scratch: ") + hipGetErrorString(e);
        return PIC_EDEVICE;
    }
    g_scratch_ptr[dev] = (unsigned char *)p;
    return PIC_OK;
}

extern "C" {

PIC_API int pic_get_particles_by_id_noalloc(pic_ctx *ctx, int32_t species, const int64_t *ids, int64_t n,
                                            double *x3, double *u3, int32_t *found) {
    if (!ctx) return PIC_EINVAL;
    if (ctx->sticky) return ctx->sticky;
    if (species < 0 || species >= ctx->nsp || n < 0 || (n > 0 && (!ids || !x3 || !u3 || !found)))
        return ctx->fail(PIC_EINVAL, "bad species, count or null arrays");
    if (n > kNoallocMaxIds)
        return ctx->fail(PIC_EINVAL, "more ids than the no-allocation lookup holds (65536)");
    if (n == 0) return PIC_OK;
    unsigned char *s = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (ctx->dev >= 0 && ctx->dev < kMaxDevices) s = g_scratch_ptr[ctx->dev];
    }
    if (!s) return ctx->fail(PIC_ESTATE, "lookup scratch not set up on this device");
    for (int64_t i = 0; i < n; ++i)
        if (ids[i] < 0) return ctx->fail(PIC_EINVAL, "negative id");
    hipStream_t st = ctx->st;
    const int ni = (int)n;
    hipError_t e = hipMemcpyAsync(s + kOffIds, ids, 8 * (size_t)n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        k_na_clear<<<(unsigned)((kSlots + 255) / 256), 256, 0, st>>>(s, ni);
        k_na_insert<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(s, ni);
        const int np = (int)ctx->np;
        if (np > 0) {
            const unsigned g = (unsigned)((np + 255) / 256);
            if (ctx->prec == 8) k_na_find<double><<<g, 256, 0, st>>>(view<double>(ctx->P[ctx->pcur]), np, species, s);
            else k_na_find<float><<<g, 256, 0, st>>>(view<float>(ctx->P[ctx->pcur]), np, species, s);
        }
        e = hipGetLastError();
    }
    int flag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(x3, s + kOffX, 24 * (size_t)n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(u3, s + kOffU, 24 * (size_t)n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(found, s + kOffFound, 4 * (size_t)n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, s + kOffFlag, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return ctx->hip_fail(e, "id lookup without allocation");
    if (flag) return ctx->fail(PIC_EINVAL, "repeated id");
    return PIC_OK;
}

}  // extern "C"
