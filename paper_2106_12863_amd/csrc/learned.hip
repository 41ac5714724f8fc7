// Learned position model over a table's interval boundaries (not in the
// paper; it only speeds up finding the interval that Algorithm 1's matching
// definition fixes).
//
// Given sorted boundaries B[0..m), a model predicts the interval j of an
// address a (B[j] <= a < B[j+1]); the measured maximum error e of the rounded
// prediction bounds a search over [p - e, p + e] whose bracket is checked, so
// lookups stay exact whatever the model's quality.
//
//   PLA: segments (knot_s, c_s, g_s) predicting j ~ c_s + g_s (a - knot_s)
//        in float32 with g_s >= 0, so the prediction is monotone inside a
//        segment and the error measured at both ends of every interval bounds
//        every address.  Either an error-bounded greedy segmentation on the
//        host (the default; it aims at a bound small enough for the window
//        search of the lookup kernels), or S equal-count segments
//        (knot_s = B[floor(s m / S)]) with least-squares lines fitted in
//        float64 on the GPU.
//   MLP: 1-16-1 ReLU network on x = a / 2^32 fitted to y = j / m by
//        full-batch Adam with this file's forward/backward kernels; it is not
//        monotone, so the bracket check and fallback keep lookups exact.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "sinet_device.h"
#include "sinet_internal.h"

namespace sinet {

constexpr int kH = 16;
constexpr int kP = SINET_MLP_PARAMS;   // 49
constexpr int kAcc = kP + 1;           // gradient + loss
constexpr int kGradBlock = 256;
constexpr int kGradBlocks = 512;

// ---------------------------------------------------------------------------
// PLA fit: one workgroup per segment, float64 centred sums.
// ---------------------------------------------------------------------------
__global__ void k_pla_fit(const uint32_t* __restrict__ B, uint32_t m, uint32_t S,
                          uint32_t* __restrict__ knot, float* __restrict__ c,
                          float* __restrict__ g) {
    __shared__ double red[2][256];
    const uint32_t s = blockIdx.x;
    const uint64_t k0 = (uint64_t)s * m / S, k1 = (uint64_t)(s + 1) * m / S;
    const uint32_t kn = B[k0];
    const double n = (double)(k1 - k0);
    // pass 1: mean of u = B[j] - knot
    double su = 0.0;
    for (uint64_t j = k0 + threadIdx.x; j < k1; j += blockDim.x) su += (double)(B[j] - kn);
    red[0][threadIdx.x] = su;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[0][threadIdx.x] += red[0][threadIdx.x + w];
        __syncthreads();
    }
    const double um = red[0][0] / n;
    const double jm = 0.5 * (double)(k0 + k1 - 1);
    __syncthreads();
    // pass 2: centred co-moments
    double suj = 0.0, suu = 0.0;
    for (uint64_t j = k0 + threadIdx.x; j < k1; j += blockDim.x) {
        double du = (double)(B[j] - kn) - um;
        suj += du * ((double)j - jm);
        suu += du * du;
    }
    red[0][threadIdx.x] = suj;
    red[1][threadIdx.x] = suu;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double slope = red[1][0] > 0.0 ? red[0][0] / red[1][0] : 0.0;
        if (!(slope > 0.0)) slope = 0.0;
        knot[s] = kn;
        g[s] = (float)slope;
        c[s] = (float)(jm - slope * um);
    }
}

// ---------------------------------------------------------------------------
// error measurement with the inference arithmetic
// ---------------------------------------------------------------------------
template <bool MLP>
__global__ void k_measure_err(DevTable t, unsigned int* __restrict__ out) {
    unsigned int worst = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < t.m; j += stride) {
        const uint32_t lo = t.B[j];
        const uint32_t hi = j + 1 < t.m ? t.B[j + 1] - 1u : 0xFFFFFFFFu;
        int p0, p1;
        if constexpr (MLP) {
            p0 = clamp_pos(mlp_predict(t.mlp, t.m_f, lo), t.m);
            p1 = clamp_pos(mlp_predict(t.mlp, t.m_f, hi), t.m);
        } else {
            p0 = clamp_pos(pla_predict(t.knot, t.pla_c, t.pla_g, t.segments, lo), t.m);
            p1 = clamp_pos(pla_predict(t.knot, t.pla_c, t.pla_g, t.segments, hi), t.m);
        }
        const int jj = (int)j;
        unsigned int e0 = (unsigned int)(p0 > jj ? p0 - jj : jj - p0);
        unsigned int e1 = (unsigned int)(p1 > jj ? p1 - jj : jj - p1);
        worst = max(worst, max(e0, e1));
    }
    // wave maximum, then one atomic per wave
    for (int o = 32; o > 0; o >>= 1) worst = max(worst, (unsigned int)__shfl_xor((int)worst, o));
    if ((threadIdx.x & 63) == 0) atomicMax(out, worst);
}

sinet_status measure_err(const DevTable& t, bool mlp, hipStream_t s, uint32_t* err) {
    unsigned int* d = nullptr;
    hipError_t e = hipMallocAsync((void**)&d, sizeof(unsigned int), s);
    if (e != hipSuccess) return check_hip(e, "error counter allocation");
    const unsigned int zero = 0;
    e = hipMemcpyAsync(d, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
    uint64_t blocks = (t.m + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (e == hipSuccess) {
        if (mlp) hipLaunchKernelGGL(k_measure_err<true>, dim3((unsigned)blocks), dim3(256), 0, s, t, d);
        else hipLaunchKernelGGL(k_measure_err<false>, dim3((unsigned)blocks), dim3(256), 0, s, t, d);
        e = hipGetLastError();
    }
    unsigned int h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(d, s);
    if (e != hipSuccess) return check_hip(e, "error measurement");
    *err = h;
    return SINET_OK;
}

// Segment directory of a PLA: for each radix bucket r (the top radix_bits
// address bits) the last segment whose knot is <= r's first address, plus a
// final entry S - 1.  The segment of an address a in bucket r is then among
// dir[r] .. dir[r + 1].  Stored as 16-bit entries, two per word.
hipError_t upload_radix(sinet_table* t, const std::vector<uint32_t>& knots) {
    const uint32_t bits = t->dev.radix_bits;
    const uint32_t nb = 1u << bits;
    std::vector<uint32_t> words(radix_words(bits), 0);
    uint32_t s = 0;
    const uint32_t S = (uint32_t)knots.size();
    for (uint32_t r = 0; r <= nb; ++r) {
        uint32_t e;
        if (r == nb) {
            e = S - 1;
        } else {
            const uint64_t first = (uint64_t)r << (32 - bits);
            while (s + 1 < S && knots[s + 1] <= first) ++s;
            e = s;
        }
        words[r >> 1] |= (e & 0xFFFFu) << ((r & 1) * 16);
    }
    return hipMemcpy((void*)t->dev.radix, words.data(), 4 * words.size(), hipMemcpyHostToDevice);
}

// Greedy error-bounded segmentation ("shrinking cone"): a segment's line
// passes through its first boundary (B[j0], j0) and keeps the interval of
// slopes that predict every later interval j of the segment within +-E at
// both of its ends, B[j] and B[j+1] - 1; when the interval of slopes
// empties, the next segment starts.  Slopes are >= 0 (the middle of the
// feasible interval), so predictions stay monotone inside a segment.
static void cone_segments(const std::vector<uint32_t>& B, double E, std::vector<uint32_t>& knot,
                          std::vector<float>& c, std::vector<float>& g) {
    knot.clear();
    c.clear();
    g.clear();
    const size_t m = B.size();
    auto end_of = [&](size_t j) { return j + 1 < m ? (double)B[j + 1] - 1.0 : 4294967295.0; };
    size_t j0 = 0;
    while (j0 < m) {
        const double x0 = B[j0], y0 = (double)j0;
        double lo = 0.0, hi = 1e300;
        const double e0 = end_of(j0) - x0;  // the first interval's own end
        if (e0 > 0) hi = E / e0;
        size_t j = j0 + 1;
        for (; j < m; ++j) {
            const double dx = (double)B[j] - x0;
            const double ex = end_of(j) - x0;
            const double nlo = std::max(lo, ((double)j - E - y0) / dx);
            const double nhi = std::min(hi, ((double)j + E - y0) / ex);
            if (nlo > nhi) break;
            lo = nlo;
            hi = nhi;
        }
        double slope = hi < 1e299 ? 0.5 * (lo + hi) : 0.0;
        if (!(slope >= 0.0)) slope = 0.0;
        knot.push_back(B[j0]);
        c.push_back((float)y0);
        g.push_back((float)slope);
        j0 = j;
    }
}

// Upload a segmentation, its radix directory, and measure its bound.
static sinet_status set_segments(sinet_table* t, const std::vector<uint32_t>& knots,
                                 const std::vector<float>& c, const std::vector<float>& g,
                                 hipStream_t s, uint32_t* err) {
    DevTable& d = t->dev;
    const uint32_t S = (uint32_t)knots.size();
    hipError_t e = hipMemcpyAsync((void*)d.knot, knots.data(), 4ull * S, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync((void*)d.pla_c, c.data(), 4ull * S, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync((void*)d.pla_g, g.data(), 4ull * S, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return check_hip(e, "PLA upload");
    d.segments = S;
    e = upload_radix(t, knots);
    if (e != hipSuccess) return check_hip(e, "PLA directory upload");
    return measure_err(d, false, s, err);
}

// S > 0: S equal-count segments fitted on the GPU.  S == 0: error-bounded
// segmentation for target E; E == 0 first tries bounds that allow the window
// search (measured max_err <= kPlaWindowErr) with at most max_window
// segments, then 8, doubled until the segments fit max_segments.
sinet_status train_pla(sinet_table* t, uint32_t S, uint32_t E, uint32_t max_segments,
                       uint32_t max_window, hipStream_t s, sinet_train_report* r) {
    DevTable& d = t->dev;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, s);
    std::vector<uint32_t> knots;
    uint32_t err = 0;
    bool window = false;
    if (S) {
        // equal-count segments, least-squares lines fitted on the GPU
        if (S > d.m) S = d.m;
        if (S > max_segments) S = max_segments;
        hipLaunchKernelGGL(k_pla_fit, dim3(S), dim3(256), 0, s, d.B, d.m, S, (uint32_t*)d.knot,
                           (float*)d.pla_c, (float*)d.pla_g);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return check_hip(e, "PLA fit");
        knots.resize(S);
        for (uint32_t k = 0; k < S; ++k) knots[k] = t->B[(uint64_t)k * d.m / S];
        d.segments = S;
        e = upload_radix(t, knots);
        if (e != hipSuccess) return check_hip(e, "PLA directory upload");
        sinet_status st = measure_err(d, false, s, &err);
        if (st != SINET_OK) return st;
        window = err <= kPlaWindowErr;
    } else {
        std::vector<float> c, g;
        bool done = false;
        if (E == 0) {
            // the float32 evaluation and rounding can add one to a cone bound
            for (double target : {6.0, 5.5, 5.0, 4.5, 4.0}) {
                cone_segments(t->B, target, knots, c, g);
                if (knots.size() > max_window) break;  // smaller targets need more
                sinet_status st = set_segments(t, knots, c, g, s, &err);
                if (st != SINET_OK) return st;
                if (err <= kPlaWindowErr) {
                    window = done = true;
                    break;
                }
            }
        }
        if (!done) {
            double target = E ? (double)E : 8.0;
            for (;;) {
                cone_segments(t->B, target, knots, c, g);
                if (knots.size() <= max_segments) break;
                target *= 2;
            }
            sinet_status st = set_segments(t, knots, c, g, s, &err);
            if (st != SINET_OK) return st;
            window = err <= kPlaWindowErr && knots.size() <= max_window;
        }
        S = (uint32_t)knots.size();
    }
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    d.max_err = err;
    d.pla_window = window ? 1u : 0u;
    t->segments = S;
    r->max_err = err;
    r->max_err_untrained = err;
    r->train_ms = ms;
    return SINET_OK;
}

// ---------------------------------------------------------------------------
// MLP forward/backward: per-block partial sums in a fixed order
// ---------------------------------------------------------------------------
// acc layout: [0..16) dL/dw1, [16..32) dL/db1, [32..48) dL/dw2, [48] dL/db2,
// [49] sum of squared residuals.  Unscaled: the caller multiplies by 2/n
// (gradient) and 1/n (loss).
__global__ void __launch_bounds__(kGradBlock)
k_mlp_partial(const float* __restrict__ w, const float* __restrict__ x,
              const float* __restrict__ y, uint64_t n, float* __restrict__ partial) {
    __shared__ float red[kAcc][kGradBlock + 1];
    float acc[kAcc];
#pragma unroll
    for (int k = 0; k < kAcc; ++k) acc[k] = 0.f;
    float w1[kH], b1[kH], w2[kH];
#pragma unroll
    for (int k = 0; k < kH; ++k) {
        w1[k] = w[k];
        b1[k] = w[kH + k];
        w2[k] = w[2 * kH + k];
    }
    const float b2 = w[3 * kH];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float xi = x[i];
        float z[kH];
        float f = b2;
#pragma unroll
        for (int k = 0; k < kH; ++k) {
            z[k] = __fadd_rn(__fmul_rn(w1[k], xi), b1[k]);
            f = __fadd_rn(f, __fmul_rn(w2[k], fmaxf(z[k], 0.f)));
        }
        const float r = f - y[i];
        acc[kP] += r * r;
        acc[3 * kH] += r;
#pragma unroll
        for (int k = 0; k < kH; ++k) {
            const float h = fmaxf(z[k], 0.f);
            acc[2 * kH + k] += r * h;
            const float dz = z[k] > 0.f ? r * w2[k] : 0.f;
            acc[kH + k] += dz;
            acc[k] += dz * xi;
        }
    }
#pragma unroll
    for (int k = 0; k < kAcc; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int wdt = kGradBlock / 2; wdt > 0; wdt >>= 1) {
        if ((int)threadIdx.x < wdt)
            for (int k = 0; k < kAcc; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + wdt];
        __syncthreads();
    }
    if ((int)threadIdx.x < kAcc) partial[(uint64_t)blockIdx.x * kAcc + threadIdx.x] = red[threadIdx.x][0];
}

// Sum the block partials (float64, fixed order), scale, and optionally apply
// one Adam step (Kingma and Ba, 2015) to w.  kFinishLanes lanes share one
// accumulator: each sums a strided slice of the blocks, then a fixed shuffle
// tree combines the slices.
constexpr int kFinishLanes = 16;

__global__ void __launch_bounds__(kAcc * kFinishLanes)
k_mlp_finish(const float* __restrict__ partial, int nblocks, double inv_n,
             float* __restrict__ w, float* __restrict__ grad_out, float* __restrict__ loss_out,
             float* __restrict__ m1, float* __restrict__ m2, int step, float lr) {
    const int k = threadIdx.x / kFinishLanes;
    const int l = threadIdx.x % kFinishLanes;
    double s = 0.0;
    for (int b = l; b < nblocks; b += kFinishLanes) s += (double)partial[(uint64_t)b * kAcc + k];
    for (int o = kFinishLanes / 2; o > 0; o >>= 1) s += __shfl_down(s, o, kFinishLanes);
    if (l != 0) return;
    if (k == kP) {
        if (loss_out) loss_out[0] = (float)(s * inv_n);
        return;
    }
    const float gk = (float)(2.0 * s * inv_n);
    if (grad_out) grad_out[k] = gk;
    if (step > 0) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float a = b1 * m1[k] + (1.f - b1) * gk;
        const float v = b2 * m2[k] + (1.f - b2) * gk * gk;
        m1[k] = a;
        m2[k] = v;
        const float mh = a / (1.f - powf(b1, (float)step));
        const float vh = v / (1.f - powf(b2, (float)step));
        w[k] -= lr * mh / (sqrtf(vh) + eps);
    }
}

__global__ void k_make_xy(const uint32_t* __restrict__ B, uint32_t m, float* __restrict__ x,
                          float* __restrict__ y) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
        x[j] = __fmul_rn(__uint2float_rn(B[j]), 2.3283064365386963e-10f);
        y[j] = (float)((double)j / (double)m);
    }
}

static int grad_blocks(uint64_t n) {
    uint64_t b = (n + kGradBlock - 1) / kGradBlock;
    return (int)(b > kGradBlocks ? kGradBlocks : (b < 1 ? 1 : b));
}

sinet_status mlp_loss_grad(const float* params, const float* x, const float* y, uint64_t n,
                           float* loss, float* grad, hipStream_t s) {
    const int nb = grad_blocks(n);
    float* partial = nullptr;
    hipError_t e = hipMallocAsync((void**)&partial, sizeof(float) * kAcc * nb, s);
    if (e != hipSuccess) return check_hip(e, "gradient workspace");
    hipLaunchKernelGGL(k_mlp_partial, dim3(nb), dim3(kGradBlock), 0, s, params, x, y, n, partial);
    e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mlp_finish, dim3(1), dim3(kAcc * kFinishLanes), 0, s, partial, nb,
                           1.0 / (double)n,
                           (float*)nullptr, grad, loss, (float*)nullptr, (float*)nullptr, 0, 0.f);
        e = hipGetLastError();
    }
    hipError_t e2 = hipFreeAsync(partial, s);
    if (e == hipSuccess) e = e2;
    return check_hip(e, "MLP gradient");
}

sinet_status train_mlp(sinet_table* t, const sinet_train_params* prm, hipStream_t s,
                       sinet_train_report* r) {
    DevTable& d = t->dev;
    const uint32_t steps = prm && prm->steps ? prm->steps : 2000;
    const float lr = prm && prm->lr > 0.f ? prm->lr : 1e-2f;
    float init[kP];
    if (prm && prm->init) {
        memcpy(init, prm->init, sizeof(init));
    } else {
        for (int k = 0; k < kH; ++k) {
            init[k] = 1.f;
            init[kH + k] = -(float)k / kH;
            init[2 * kH + k] = 0.f;
        }
        init[3 * kH] = 0.f;
    }
    const uint64_t m = d.m;
    const int nb = grad_blocks(m);
    float *x = nullptr, *y = nullptr, *partial = nullptr, *state = nullptr, *lossd = nullptr;
    hipError_t e = hipMallocAsync((void**)&x, 4 * m, s);
    if (e == hipSuccess) e = hipMallocAsync((void**)&y, 4 * m, s);
    if (e == hipSuccess) e = hipMallocAsync((void**)&partial, sizeof(float) * kAcc * nb, s);
    if (e == hipSuccess) e = hipMallocAsync((void**)&state, sizeof(float) * 2 * kP, s);
    if (e == hipSuccess) e = hipMallocAsync((void**)&lossd, sizeof(float) * 2, s);
    if (e != hipSuccess) return check_hip(e, "MLP training workspace");
    std::vector<float> zeros(2 * kP, 0.f);
    float* w = (float*)d.mlp;
    e = hipMemcpyAsync(w, init, sizeof(init), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(state, zeros.data(), sizeof(float) * 2 * kP, hipMemcpyHostToDevice, s);
    uint32_t err0 = 0;
    if (e == hipSuccess) {
        sinet_status st = measure_err(d, true, s, &err0);
        if (st != SINET_OK) return st;
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, s);
    if (e == hipSuccess) {
        uint64_t blocks = (m + 255) / 256;
        hipLaunchKernelGGL(k_make_xy, dim3((unsigned)(blocks > 4096 ? 4096 : blocks)), dim3(256), 0,
                           s, d.B, d.m, x, y);
        e = hipGetLastError();
    }
    for (uint32_t it = 1; e == hipSuccess && it <= steps + 1; ++it) {
        hipLaunchKernelGGL(k_mlp_partial, dim3(nb), dim3(kGradBlock), 0, s, (const float*)w, x, y, m,
                           partial);
        // the last launch only evaluates the final loss (no step)
        const bool last = it == steps + 1;
        float* lo = it == 1 ? lossd : (last ? lossd + 1 : nullptr);
        hipLaunchKernelGGL(k_mlp_finish, dim3(1), dim3(kAcc * kFinishLanes), 0, s, partial, nb,
                           1.0 / (double)m, w,
                           (float*)nullptr, lo, state, state + kP, last ? 0 : (int)it, lr);
        e = hipGetLastError();
    }
    (void)hipEventRecord(e1, s);
    float lh[2] = {0.f, 0.f};
    if (e == hipSuccess) e = hipMemcpyAsync(lh, lossd, sizeof(lh), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFreeAsync(x, s);
    (void)hipFreeAsync(y, s);
    (void)hipFreeAsync(partial, s);
    (void)hipFreeAsync(state, s);
    (void)hipFreeAsync(lossd, s);
    if (e != hipSuccess) return check_hip(e, "MLP training");
    uint32_t err = 0;
    sinet_status st = measure_err(d, true, s, &err);
    if (st != SINET_OK) return st;
    d.max_err = err;
    r->loss_first = lh[0];
    r->loss_last = lh[1];
    r->max_err_untrained = err0;
    r->max_err = err;
    r->train_ms = ms;
    return SINET_OK;
}

}  // namespace sinet
