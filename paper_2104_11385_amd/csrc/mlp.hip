// Learned per-box cost model: a 16-64-64-1 ReLU perceptron that predicts the
// log of a box's device-timer cycles from box features, trained and run on
// the device.  Matrix products use the bf16 matrix cores
// (v_mfma_f32_16x16x16bf16_1k) with fp32 accumulation; master weights, biases,
// the loss and Adam run in fp32.  It replaces neither measurement: the timer
// judges it and the particle+cell heuristic is its fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "runtime.hpp"

namespace pb {

constexpr int NI = 16, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NI, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;

struct MlpState {
    float *P = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
    float *mean = nullptr, *istd = nullptr;   // standardisation: (x - mean) * istd
    float *loss = nullptr;
    float *X = nullptr, *y = nullptr, *yhat = nullptr;
    int *perm = nullptr;
    int64_t cap = 0;
    float h_mean[NI], h_std[NI];  // std 0: a feature constant in training, ignored
    // target transform: with base = 1 the network models the residual
    // r = y - ln(1 + N) (N = the box's particles, from features 0 and 1),
    // else r = y; it is trained on (r - ymean) / ystd and predicts
    // r = ymean + ystd * output; [ymin, ymax] is the training residuals'
    // range, to which learned costs clamp r (ymin > ymax: no clamp)
    float ymean = 0.f, ystd = 1.f, ymin = 1.f, ymax = 0.f, base = 0.f;
    bool ready = false;
    int64_t t = 0;
};

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// fp32 -> bf16, round to nearest even
__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// Operand fetch for the 16x16x16 bf16 matrix instruction.  Lane l supplies
// A[l%16][k0 + 4(l/16) + t] and B[k0 + 4(l/16) + t][l%16], t = 0..3, and
// receives D[4(l/16) + t][l%16].
// A[m][k] = src[m][k] (row-major, leading dimension ld)
__device__ __forceinline__ bf16x4 ldA_rows(const unsigned short *src, int ld, int m0, int k0) {
    int l = threadIdx.x & 63;
    const unsigned short *p = src + (m0 + (l & 15)) * ld + k0 + 4 * (l >> 4);
    bf16x4 r;
    for (int t = 0; t < 4; ++t) r[t] = (short)p[t];
    return r;
}
// A[m][k] = src[k][m]
__device__ __forceinline__ bf16x4 ldA_cols(const unsigned short *src, int ld, int m0, int k0) {
    int l = threadIdx.x & 63;
    bf16x4 r;
    for (int t = 0; t < 4; ++t) r[t] = (short)src[(k0 + 4 * (l >> 4) + t) * ld + m0 + (l & 15)];
    return r;
}
// B[k][n] = src[n][k]
__device__ __forceinline__ bf16x4 ldB_rows(const unsigned short *src, int ld, int n0, int k0) {
    int l = threadIdx.x & 63;
    const unsigned short *p = src + (n0 + (l & 15)) * ld + k0 + 4 * (l >> 4);
    bf16x4 r;
    for (int t = 0; t < 4; ++t) r[t] = (short)p[t];
    return r;
}
// B[k][n] = src[k][n]
__device__ __forceinline__ bf16x4 ldB_cols(const unsigned short *src, int ld, int n0, int k0) {
    int l = threadIdx.x & 63;
    bf16x4 r;
    for (int t = 0; t < 4; ++t) r[t] = (short)src[(k0 + 4 * (l >> 4) + t) * ld + n0 + (l & 15)];
    return r;
}
__device__ __forceinline__ f32x4 mma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

struct WaveBuf {  // per-wave scratch for one 16-sample tile
    unsigned short xb[16 * NI];
    unsigned short h1b[16 * NH], h2b[16 * NH], dz2b[16 * NH], dz1b[16 * NH];
    float h1f[16 * NH], h2f[16 * NH];
    float dy[16];
    float colsum[NH];
};

struct FbArgs {
    const float *X;      // [n][16] raw features
    const float *y;      // [n] targets (nullable for prediction)
    const int *rows;     // sample indices (nullable: identity)
    int nrows;           // samples in this call
    const float *mean, *istd;
    const float *P;
    float *g;            // gradient accumulator (nullable: forward only)
    float *loss;         // sum of squared errors (nullable)
    float *yhat;         // predictions (nullable), indexed like rows
    float scale;         // d loss / d yhat = scale * (yhat - y)
};

// Forward (+ backward) over nrows samples.  Blocks of 4 waves; every wave of
// a block runs the same number of tiles so block barriers are uniform.
__global__ __launch_bounds__(256) void k_mlp(FbArgs A) {
    __shared__ unsigned short w1b[NH * NI], w2b[NH * NH];
    __shared__ float w3f[NH], b1[NH], b2[NH];
    __shared__ WaveBuf wb[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < NH * NI; i += 256) w1b[i] = f2bf(A.P[OFF_W1 + i]);
    for (int i = tid; i < NH * NH; i += 256) w2b[i] = f2bf(A.P[OFF_W2 + i]);
    if (tid < NH) {
        w3f[tid] = bf2f(f2bf(A.P[OFF_W3 + tid]));
        b1[tid] = A.P[OFF_B1 + tid];
        b2[tid] = A.P[OFF_B2 + tid];
    }
    const float b3 = A.P[OFF_B3];
    __syncthreads();
    WaveBuf &W = wb[wave];
    const bool back = A.g != nullptr;

    f32x4 gW2[4][4], gW1[4];
    for (int a = 0; a < 4; ++a) {
        gW1[a] = f32x4{0, 0, 0, 0};
        for (int b = 0; b < 4; ++b) gW2[a][b] = f32x4{0, 0, 0, 0};
    }
    float gW3 = 0.f, gB1 = 0.f, gB2 = 0.f, gB3 = 0.f;

    const int ntiles = (A.nrows + 15) / 16;
    const int groups = (ntiles + 4 * gridDim.x - 1) / (4 * gridDim.x);
    for (int grp = 0; grp < groups; ++grp) {
        int tile = (grp * gridDim.x + blockIdx.x) * 4 + wave;
        int r0 = tile * 16;
        int nvalid = max(0, min(16, A.nrows - r0));
        // standardised bf16 inputs
        for (int q = lane; q < 16 * NI; q += 64) {
            int s = q / NI, i = q % NI;
            float x = 0.f;
            if (s < nvalid) {
                int row = A.rows ? A.rows[r0 + s] : r0 + s;
                x = (A.X[(size_t)row * NI + i] - A.mean[i]) * A.istd[i];
            }
            W.xb[q] = f2bf(x);
        }
        __syncthreads();
        // layer 1: Z1 = X W1^T + b1 (K = 16)
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 acc = {0, 0, 0, 0};
            acc = mma(ldA_rows(W.xb, NI, 0, 0), ldB_rows(w1b, NI, nt * 16, 0), acc);
            for (int t = 0; t < 4; ++t) {
                int s = 4 * (lane >> 4) + t, o = nt * 16 + (lane & 15);
                float z = acc[t] + b1[o];
                float h = z > 0.f ? z : 0.f;
                W.h1f[s * NH + o] = h;
                W.h1b[s * NH + o] = f2bf(h);
            }
        }
        __syncthreads();
        // layer 2: Z2 = H1 W2^T + b2 (K = 64)
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 acc = {0, 0, 0, 0};
            for (int kt = 0; kt < 4; ++kt)
                acc = mma(ldA_rows(W.h1b, NH, 0, kt * 16), ldB_rows(w2b, NH, nt * 16, kt * 16), acc);
            for (int t = 0; t < 4; ++t) {
                int s = 4 * (lane >> 4) + t, o = nt * 16 + (lane & 15);
                float z = acc[t] + b2[o];
                float h = z > 0.f ? z : 0.f;
                W.h2f[s * NH + o] = h;
                W.h2b[s * NH + o] = f2bf(h);
            }
        }
        __syncthreads();
        // layer 3 and the output gradient
        if (lane < 16) {
            float out = 0.f;
            for (int k = 0; k < NH; ++k) out += bf2f(W.h2b[lane * NH + k]) * w3f[k];
            out += b3;
            float dy = 0.f;
            if (lane < nvalid) {
                int row = A.rows ? A.rows[r0 + lane] : r0 + lane;
                if (A.yhat) A.yhat[r0 + lane] = out;
                if (A.y) {
                    float r = out - A.y[row];
                    dy = A.scale * r;
                    if (A.loss) atomicAdd(A.loss, r * r);
                }
                (void)row;
            }
            W.dy[lane] = dy;
        }
        __syncthreads();
        if (!back) continue;
        // dW3, db3; dZ2 = dy W3 * [Z2 > 0]
        {
            float s3 = 0.f;
            for (int s = 0; s < 16; ++s) s3 += W.dy[s] * bf2f(W.h2b[s * NH + lane]);
            gW3 += s3;
            if (lane == 0)
                for (int s = 0; s < 16; ++s) gB3 += W.dy[s];
            float cs = 0.f;
            for (int s = 0; s < 16; ++s) {
                float d = W.h2f[s * NH + lane] > 0.f ? W.dy[s] * w3f[lane] : 0.f;
                cs += d;
                W.dz2b[s * NH + lane] = f2bf(d);
            }
            gB2 += cs;
        }
        __syncthreads();
        // dW2 += dZ2^T H1 (K = 16 samples)
        for (int mt = 0; mt < 4; ++mt)
            for (int nt = 0; nt < 4; ++nt)
                gW2[mt][nt] = mma(ldA_cols(W.dz2b, NH, mt * 16, 0), ldB_cols(W.h1b, NH, nt * 16, 0), gW2[mt][nt]);
        // dH1 = dZ2 W2 (K = 64); dZ1 = dH1 * [Z1 > 0]
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 acc = {0, 0, 0, 0};
            for (int kt = 0; kt < 4; ++kt)
                acc = mma(ldA_rows(W.dz2b, NH, 0, kt * 16), ldB_cols(w2b, NH, nt * 16, kt * 16), acc);
            for (int t = 0; t < 4; ++t) {
                int s = 4 * (lane >> 4) + t, i = nt * 16 + (lane & 15);
                float d = W.h1f[s * NH + i] > 0.f ? acc[t] : 0.f;
                W.h1f[s * NH + i] = d;  // reuse as dZ1 (fp32) for the bias gradient
                W.dz1b[s * NH + i] = f2bf(d);
            }
        }
        __syncthreads();
        {
            float cs = 0.f;
            for (int s = 0; s < 16; ++s) cs += W.h1f[s * NH + lane];
            gB1 += cs;
        }
        // dW1 += dZ1^T X (K = 16 samples)
        for (int mt = 0; mt < 4; ++mt) gW1[mt] = mma(ldA_cols(W.dz1b, NH, mt * 16, 0), ldB_cols(W.xb, NI, 0, 0), gW1[mt]);
        __syncthreads();
    }
    if (!back) return;
    for (int mt = 0; mt < 4; ++mt)
        for (int t = 0; t < 4; ++t) {
            int o = mt * 16 + 4 * (lane >> 4) + t;
            atomicAdd(&A.g[OFF_W1 + o * NI + (lane & 15)], gW1[mt][t]);
            for (int nt = 0; nt < 4; ++nt) atomicAdd(&A.g[OFF_W2 + o * NH + nt * 16 + (lane & 15)], gW2[mt][nt][t]);
        }
    atomicAdd(&A.g[OFF_W3 + lane], gW3);
    atomicAdd(&A.g[OFF_B1 + lane], gB1);
    atomicAdd(&A.g[OFF_B2 + lane], gB2);
    if (lane == 0) atomicAdd(&A.g[OFF_B3], gB3);
}

__global__ void k_adam(float *P, float *g, float *m, float *v, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    g[i] = 0.f;
}

__global__ void k_zero(float *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

static unsigned mlp_blocks(int nrows) {
    int ntiles = (nrows + 15) / 16;
    int b = (ntiles + 3) / 4;
    return (unsigned)std::max(1, std::min(b, 256));
}

}  // namespace pb

using namespace pb;

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {

uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
double unit(uint64_t &s) { return (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace

#define MLPC(expr)                                        \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return ctx->hip_fail(e_, #expr); \
    } while (0)

static int mlp_ensure(pic_ctx *ctx, int64_t n) {
    if (!ctx->mlp) {
        ctx->mlp = new MlpState();
        MlpState &M = *ctx->mlp;
        int rc;
        if ((rc = ctx->dalloc((void **)&M.P, 4 * NPARAM)) || (rc = ctx->dalloc((void **)&M.m, 4 * NPARAM)) ||
            (rc = ctx->dalloc((void **)&M.v, 4 * NPARAM)) || (rc = ctx->dalloc((void **)&M.g, 4 * NPARAM)) ||
            (rc = ctx->dalloc((void **)&M.mean, 4 * NI)) || (rc = ctx->dalloc((void **)&M.istd, 4 * NI)) ||
            (rc = ctx->dalloc((void **)&M.loss, 4)))
            return rc;
        for (int i = 0; i < NI; ++i) {
            M.h_mean[i] = 0.f;
            M.h_std[i] = 1.f;
        }
    }
    MlpState &M = *ctx->mlp;
    if (n > M.cap) {
        int rc;
        if ((rc = ctx->dalloc((void **)&M.X, 4 * NI * (size_t)n)) || (rc = ctx->dalloc((void **)&M.y, 4 * (size_t)n)) ||
            (rc = ctx->dalloc((void **)&M.yhat, 4 * (size_t)n)) || (rc = ctx->dalloc((void **)&M.perm, 4 * (size_t)n)))
            return rc;
        M.cap = n;
    }
    return PIC_OK;
}

static int mlp_upload_norm(pic_ctx *ctx) {
    MlpState &M = *ctx->mlp;
    float istd[NI];
    for (int i = 0; i < NI; ++i) istd[i] = M.h_std[i] > 0.f ? 1.f / M.h_std[i] : 0.f;
    MLPC(hipMemcpyAsync(M.mean, M.h_mean, 4 * NI, hipMemcpyHostToDevice, ctx->st));
    MLPC(hipMemcpyAsync(M.istd, istd, 4 * NI, hipMemcpyHostToDevice, ctx->st));
    return PIC_OK;
}

// ln(1 + N) of a box from its raw features 0 and 1 (ln(1 + N_s) of the
// first two species).
static double ln1p_particles(const float *x) {
    double ne = std::max(0.0, std::expm1((double)x[0])), ni = std::max(0.0, std::expm1((double)x[1]));
    return std::log1p(ne + ni);
}

static int mlp_forward(pic_ctx *ctx, const float *dX, int64_t n, float *dyhat) {
    MlpState &M = *ctx->mlp;
    FbArgs A{};
    A.X = dX;
    A.nrows = (int)n;
    A.mean = M.mean;
    A.istd = M.istd;
    A.P = M.P;
    A.yhat = dyhat;
    k_mlp<<<mlp_blocks((int)n), 256, 0, ctx->st>>>(A);
    MLPC(hipGetLastError());
    return PIC_OK;
}

// Predicted cycles max(0, exp(yhat) - 1) of every box (the model is trained on
// ln(1 + cycles) so that boxes without work are represented); falls back to
// the heuristic when no model is loaded, or when the prediction made for the
// interval just measured missed the measured timer costs by more than 15%
// relative error, sum_b |pred_b s - t_b| / sum_b t_b with the prediction
// scaled to the measured total, s = sum t / sum pred.  Errors are weighted
// by cost, so that a box holding a few stray particles cannot trigger the
// fallback alone, and a common factor (a clock rate that differs from the
// training runs') does not count: mappings and E depend only on cost ratios.
int pic_ctx::learned_costs(double *costs, int *used) {
    *used = PIC_COST_HEURISTIC;
    if (!mlp || !mlp->ready) return PIC_OK;
    bool fallback = false;
    if (last_pred.size() == (size_t)nb && last_timer.size() == (size_t)nb) {
        double ps = 0.0, tot = 0.0;
        for (int b = 0; b < nb; ++b) {
            ps += last_pred[b];
            tot += last_timer[b];
        }
        if (tot > 0.0 && ps > 0.0) {
            const double sc = tot / ps;
            double err = 0.0;
            for (int b = 0; b < nb; ++b) err += std::fabs(last_pred[b] * sc - last_timer[b]);
            mare = err / tot;
        } else {
            mare = (tot > 0.0) != (ps > 0.0) ? 1.0 : 0.0;
        }
        fallback = mare > 0.15;
    }
    int rc = features_device();
    if (rc) return rc;
    if ((rc = mlp_ensure(this, nb))) return rc;
    if ((rc = mlp_upload_norm(this))) return rc;
    if ((rc = mlp_forward(this, d_feat, nb, mlp->yhat))) return rc;
    std::vector<float> yh(nb), feat((size_t)nb * NI);
    hipError_t e = hipMemcpyAsync(yh.data(), mlp->yhat, 4 * (size_t)nb, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(feat.data(), d_feat, 4 * (size_t)nb * NI, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "learned costs");
    last_pred.resize(nb);
    const MlpState &M = *mlp;
    for (int b = 0; b < nb; ++b) {
        // back to ln(1 + cycles), the residual clamped to the range the model
        // was trained on
        double r = (double)M.ymean + (double)M.ystd * (double)yh[b];
        if (M.ymin <= M.ymax) r = std::min(std::max(r, (double)M.ymin), (double)M.ymax);
        const double y = r + (M.base != 0.f ? ln1p_particles(&feat[(size_t)b * NI]) : 0.0);
        last_pred[b] = std::max(0.0, std::expm1(y));
    }
    if (fallback) return PIC_OK;
    for (int b = 0; b < nb; ++b) costs[b] = last_pred[b];
    *used = PIC_COST_LEARNED;
    return PIC_OK;
}

void pic_ctx::mlp_release() {
    delete mlp;
    mlp = nullptr;
}

extern "C" {

PIC_API int32_t pic_mlp_nparam(void) { return NPARAM; }

PIC_API int pic_mlp_train(pic_ctx *ctx, const float *X, const float *y, int64_t n, int32_t epochs, int32_t batch,
                          const int32_t *perm, const float *init_w, uint64_t seed, float *loss_per_epoch) {
    if (!ctx) return PIC_EINVAL;
    if (ctx->sticky) return ctx->sticky;
    if (!X || !y || n < 1 || n > INT32_MAX / NI || epochs < 0 || batch < 1)
        return ctx->fail(PIC_EINVAL, "bad training arguments");
    int rc;
    if ((rc = mlp_ensure(ctx, n))) return rc;
    MlpState &M = *ctx->mlp;
    // standardisation from the training set; a feature that is constant in
    // it gets std 0 (standardised input 0 whatever its value, so that a
    // weight it never trained cannot act on new data)
    for (int i = 0; i < NI; ++i) {
        double s = 0.0, s2 = 0.0;
        for (int64_t r = 0; r < n; ++r) s += X[r * NI + i];
        double mu = s / (double)n;
        for (int64_t r = 0; r < n; ++r) {
            double d = X[r * NI + i] - mu;
            s2 += d * d;
        }
        double sd = std::sqrt(s2 / (double)n);
        M.h_mean[i] = (float)mu;
        M.h_std[i] = sd > 1e-6 ? (float)sd : 0.f;
    }
    // The network models the residual r = y - ln(1 + N): the log of a box's
    // cycles per particle, whose spread is far narrower than that of the
    // cycles themselves (the heaviest boxes, which decide the balance, are
    // then fitted as well as the light ones).  The residuals are
    // standardised, so that the bf16 layers produce an output of order one.
    std::vector<float> ys(n);
    {
        std::vector<double> res(n);
        for (int64_t r = 0; r < n; ++r) res[r] = (double)y[r] - ln1p_particles(X + r * NI);
        double s = 0.0, s2 = 0.0, lo = res[0], hi = res[0];
        for (int64_t r = 0; r < n; ++r) {
            s += res[r];
            lo = std::min(lo, res[r]);
            hi = std::max(hi, res[r]);
        }
        double mu = s / (double)n;
        for (int64_t r = 0; r < n; ++r) s2 += (res[r] - mu) * (res[r] - mu);
        double sd = std::sqrt(s2 / (double)n);
        M.ymean = (float)mu;
        M.ystd = sd > 1e-6 ? (float)sd : 1.f;
        M.ymin = (float)lo;
        M.ymax = (float)hi;
        M.base = 1.f;
        for (int64_t r = 0; r < n; ++r) ys[r] = (float)((res[r] - mu) / (double)M.ystd);
    }
    if ((rc = mlp_upload_norm(ctx))) return rc;
    // initial weights: given, or Kaiming-uniform (biases zero)
    std::vector<float> P0(NPARAM, 0.f);
    if (init_w) {
        std::memcpy(P0.data(), init_w, 4 * NPARAM);
    } else {
        uint64_t s = seed;
        auto fill = [&](int off, int count, int fan_in) {
            double lim = std::sqrt(6.0 / fan_in);
            for (int i = 0; i < count; ++i) P0[off + i] = (float)((2.0 * unit(s) - 1.0) * lim);
        };
        fill(OFF_W1, NH * NI, NI);
        fill(OFF_W2, NH * NH, NH);
        fill(OFF_W3, NH, NH);
    }
    MLPC(hipMemcpyAsync(M.P, P0.data(), 4 * NPARAM, hipMemcpyHostToDevice, ctx->st));
    k_zero<<<(NPARAM + 255) / 256, 256, 0, ctx->st>>>(M.m, NPARAM);
    k_zero<<<(NPARAM + 255) / 256, 256, 0, ctx->st>>>(M.v, NPARAM);
    k_zero<<<(NPARAM + 255) / 256, 256, 0, ctx->st>>>(M.g, NPARAM);
    MLPC(hipMemcpyAsync(M.X, X, 4 * NI * (size_t)n, hipMemcpyHostToDevice, ctx->st));
    MLPC(hipMemcpyAsync(M.y, ys.data(), 4 * (size_t)n, hipMemcpyHostToDevice, ctx->st));
    M.t = 0;
    const float lr = 1e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    std::vector<int32_t> order(n);
    uint64_t shuf = seed ^ 0xA5A5A5A5ULL;
    for (int ep = 0; ep < epochs; ++ep) {
        if (perm) {
            std::memcpy(order.data(), perm + (size_t)ep * n, 4 * (size_t)n);
        } else {
            std::iota(order.begin(), order.end(), 0);
            for (int64_t i = n - 1; i > 0; --i) std::swap(order[i], order[(int64_t)(unit(shuf) * (double)(i + 1))]);
        }
        for (int64_t i = 0; i < n; ++i)
            if (order[i] < 0 || order[i] >= n) return ctx->fail(PIC_EINVAL, "perm entry out of range");
        MLPC(hipMemcpyAsync(M.perm, order.data(), 4 * (size_t)n, hipMemcpyHostToDevice, ctx->st));
        k_zero<<<1, 64, 0, ctx->st>>>(M.loss, 1);
        for (int64_t b0 = 0; b0 < n; b0 += batch) {
            int bs = (int)std::min<int64_t>(batch, n - b0);
            FbArgs A{};
            A.X = M.X;
            A.y = M.y;
            A.rows = M.perm + b0;
            A.nrows = bs;
            A.mean = M.mean;
            A.istd = M.istd;
            A.P = M.P;
            A.g = M.g;
            A.loss = M.loss;
            A.scale = 2.f / (float)bs;
            k_mlp<<<mlp_blocks(bs), 256, 0, ctx->st>>>(A);
            ++M.t;
            float c1 = 1.f - std::pow(b1, (float)M.t), c2 = 1.f - std::pow(b2, (float)M.t);
            k_adam<<<(NPARAM + 255) / 256, 256, 0, ctx->st>>>(M.P, M.g, M.m, M.v, lr, b1, b2, eps, c1, c2);
        }
        MLPC(hipGetLastError());
        if (loss_per_epoch) {
            float l = 0.f;
            MLPC(hipMemcpyAsync(&l, M.loss, 4, hipMemcpyDeviceToHost, ctx->st));
            MLPC(hipStreamSynchronize(ctx->st));
            loss_per_epoch[ep] = l / (float)n * M.ystd * M.ystd;  // in units of y (= of r)
        }
    }
    MLPC(hipStreamSynchronize(ctx->st));
    M.ready = true;
    ctx->last_pred.clear();
    return PIC_OK;
}

PIC_API int pic_mlp_predict(pic_ctx *ctx, const float *X, int64_t n, float *yhat) {
    if (!ctx) return PIC_EINVAL;
    if (ctx->sticky) return ctx->sticky;
    if (!X || !yhat || n < 1 || n > INT32_MAX / NI) return ctx->fail(PIC_EINVAL, "bad prediction arguments");
    if (!ctx->mlp || !ctx->mlp->ready) return ctx->fail(PIC_ESTATE, "no trained or loaded model");
    int rc;
    if ((rc = mlp_ensure(ctx, n))) return rc;
    MlpState &M = *ctx->mlp;
    if ((rc = mlp_upload_norm(ctx))) return rc;
    MLPC(hipMemcpyAsync(M.X, X, 4 * NI * (size_t)n, hipMemcpyHostToDevice, ctx->st));
    if ((rc = mlp_forward(ctx, M.X, n, M.yhat))) return rc;
    MLPC(hipMemcpyAsync(yhat, M.yhat, 4 * (size_t)n, hipMemcpyDeviceToHost, ctx->st));
    MLPC(hipStreamSynchronize(ctx->st));
    if (M.ymean != 0.f || M.ystd != 1.f || M.base != 0.f)
        for (int64_t r = 0; r < n; ++r)
            yhat[r] = (float)((double)M.ymean + (double)M.ystd * (double)yhat[r] +
                              (M.base != 0.f ? ln1p_particles(X + r * NI) : 0.0));
    return PIC_OK;
}

PIC_API int pic_mlp_loss_grad(pic_ctx *ctx, const float *X, const float *y, int64_t n, float *loss, float *grad) {
    if (!ctx) return PIC_EINVAL;
    if (ctx->sticky) return ctx->sticky;
    if (!X || !y || n < 1 || n > INT32_MAX / NI) return ctx->fail(PIC_EINVAL, "bad arguments");
    if (!ctx->mlp) return ctx->fail(PIC_ESTATE, "no weights: call pic_mlp_set_weights first");
    int rc;
    if ((rc = mlp_ensure(ctx, n))) return rc;
    MlpState &M = *ctx->mlp;
    // inputs are taken as standardised: identity transform
    float zero[NI], one[NI];
    for (int i = 0; i < NI; ++i) {
        zero[i] = 0.f;
        one[i] = 1.f;
    }
    MLPC(hipMemcpyAsync(M.mean, zero, 4 * NI, hipMemcpyHostToDevice, ctx->st));
    MLPC(hipMemcpyAsync(M.istd, one, 4 * NI, hipMemcpyHostToDevice, ctx->st));
    MLPC(hipMemcpyAsync(M.X, X, 4 * NI * (size_t)n, hipMemcpyHostToDevice, ctx->st));
    MLPC(hipMemcpyAsync(M.y, y, 4 * (size_t)n, hipMemcpyHostToDevice, ctx->st));
    k_zero<<<(NPARAM + 255) / 256, 256, 0, ctx->st>>>(M.g, NPARAM);
    k_zero<<<1, 64, 0, ctx->st>>>(M.loss, 1);
    FbArgs A{};
    A.X = M.X;
    A.y = M.y;
    A.nrows = (int)n;
    A.mean = M.mean;
    A.istd = M.istd;
    A.P = M.P;
    A.g = M.g;
    A.loss = M.loss;
    A.scale = 2.f / (float)n;
    k_mlp<<<mlp_blocks((int)n), 256, 0, ctx->st>>>(A);
    MLPC(hipGetLastError());
    float l = 0.f;
    if (grad) MLPC(hipMemcpyAsync(grad, M.g, 4 * NPARAM, hipMemcpyDeviceToHost, ctx->st));
    MLPC(hipMemcpyAsync(&l, M.loss, 4, hipMemcpyDeviceToHost, ctx->st));
    MLPC(hipStreamSynchronize(ctx->st));
    if (loss) *loss = l / (float)n;
    // restore the model's own standardisation
    return mlp_upload_norm(ctx);
}

PIC_API int pic_mlp_set_weights(pic_ctx *ctx, const float *w, int64_t n) {
    if (!ctx) return PIC_EINVAL;
    if (ctx->sticky) return ctx->sticky;
    if (!w || (n != NPARAM && n != NPARAM + 2 * NI && n != NPARAM + 2 * NI + 5))
        return ctx->fail(PIC_EINVAL, "expected nparam, nparam+32 or nparam+37 floats");
    if (n == NPARAM + 2 * NI + 5 && !(w[NPARAM + 2 * NI + 1] > 0.f))
        return ctx->fail(PIC_EINVAL, "target std must be positive");
    int rc;
    if ((rc = mlp_ensure(ctx, 1))) return rc;
    MlpState &M = *ctx->mlp;
    if (n >= NPARAM + 2 * NI) {
        for (int i = 0; i < NI; ++i) {
            M.h_mean[i] = w[NPARAM + i];
            M.h_std[i] = w[NPARAM + NI + i] > 0.f ? w[NPARAM + NI + i] : 0.f;
        }
    }
    M.ymean = 0.f;
    M.ystd = 1.f;
    M.ymin = 1.f;
    M.ymax = 0.f;
    M.base = 0.f;
    if (n == NPARAM + 2 * NI + 5) {
        M.ymean = w[NPARAM + 2 * NI];
        M.ystd = w[NPARAM + 2 * NI + 1];
        M.ymin = w[NPARAM + 2 * NI + 2];
        M.ymax = w[NPARAM + 2 * NI + 3];
        M.base = w[NPARAM + 2 * NI + 4] != 0.f ? 1.f : 0.f;
    }
    MLPC(hipMemcpyAsync(M.P, w, 4 * NPARAM, hipMemcpyHostToDevice, ctx->st));
    if ((rc = mlp_upload_norm(ctx))) return rc;
    MLPC(hipStreamSynchronize(ctx->st));
    M.ready = true;
    ctx->last_pred.clear();
    return PIC_OK;
}

PIC_API int pic_mlp_get_weights(pic_ctx *ctx, float *w, int64_t n) {
    if (!ctx) return PIC_EINVAL;
    if (ctx->sticky) return ctx->sticky;
    if (!w || n < NPARAM + 2 * NI) return ctx->fail(PIC_EINVAL, "need nparam+32 floats");
    if (!ctx->mlp) return ctx->fail(PIC_ESTATE, "no model");
    MlpState &M = *ctx->mlp;
    MLPC(hipMemcpyAsync(w, M.P, 4 * NPARAM, hipMemcpyDeviceToHost, ctx->st));
    MLPC(hipStreamSynchronize(ctx->st));
    for (int i = 0; i < NI; ++i) {
        w[NPARAM + i] = M.h_mean[i];
        w[NPARAM + NI + i] = M.h_std[i];
    }
    if (n >= NPARAM + 2 * NI + 5) {
        w[NPARAM + 2 * NI] = M.ymean;
        w[NPARAM + 2 * NI + 1] = M.ystd;
        w[NPARAM + 2 * NI + 2] = M.ymin;
        w[NPARAM + 2 * NI + 3] = M.ymax;
        w[NPARAM + 2 * NI + 4] = M.base;
    }
    return PIC_OK;
}

}  // extern "C"
