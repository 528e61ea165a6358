// rdl_train.hip -- FP32 training kernels of the learned mantissa estimator
// (an extension beyond the paper, whose estimator needs no learning).
//
// The float model mirrors the int8 one: inputs x = (S - 128)/128 for the 3x3
// x 3-channel neighbourhood, a per-exponent-bin bias row in the first layer,
// two ReLU layers of 32, three outputs predicting M / 256.  Loss: mean squared
// error.  Gradients are summed per workgroup in a fixed order, written as
// partials, and reduced in a fixed order by the Adam kernel, so a step is
// deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rdl_internal.h"

#pragma clang fp contract(off)

namespace rdl {

// Flat parameter layout (floats).
constexpr int P_W1 = 0;           // [32][27]
constexpr int P_B1 = 864;         // [32 bins][32]
constexpr int P_W2 = 1888;        // [32][32]
constexpr int P_B2 = 2912;        // [32]
constexpr int P_W3 = 2944;        // [3][32]
constexpr int P_B3 = 3040;        // [3]
constexpr int NPARAM = 3043;
constexpr int TS = 64;            // samples per workgroup per step

// One training sample: 27 feature bytes (S - 128), the exponent bin, the three
// mantissas, one pad byte.
struct Sample {
    int8_t f[27];
    uint8_t bin;
    uint8_t m[3];
    uint8_t pad;
};

__global__ __launch_bounds__(256) void k_train_samples(const uint8_t *__restrict__ rgbe, const uint8_t *__restrict__ sdr,
                                                       int H, int W, int k_img, const int64_t *__restrict__ idx,
                                                       int64_t n, Sample *__restrict__ out) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const int64_t p = idx[s];
    if (p < 0 || p >= (int64_t)H * W) return;
    const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
    Sample r;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int yy = min(max(y + k / 3 - 1, 0), H - 1), xx = min(max(x + k % 3 - 1, 0), W - 1);
        const uint8_t *q = sdr + 3 * ((int64_t)yy * W + xx);
#pragma unroll
        for (int c = 0; c < 3; ++c) r.f[3 * k + c] = (int8_t)((int)q[c] - 128);
    }
    const uint8_t *w = rgbe + 4 * p;
    r.bin = (uint8_t)min(max((int)w[3] - 136 + k_img + 24, 0), 31);
    r.m[0] = w[0];
    r.m[1] = w[1];
    r.m[2] = w[2];
    r.pad = 0;
    out[s] = r;
}

// Forward + backward of TS samples per workgroup; partial gradient sums
// part[blockIdx.x][NPARAM] and partial loss sums ploss[blockIdx.x].
__global__ __launch_bounds__(256) void k_train_grad(const float *__restrict__ prm, const Sample *__restrict__ smp,
                                                    int64_t base, int64_t n, float inv_count,
                                                    float *__restrict__ part, float *__restrict__ ploss) {
    __shared__ float w[NPARAM + 1];
    __shared__ float sx[TS][28], sa1[TS][32], sa2[TS][32], sd1[TS][32], sd2[TS][32], sdo[TS][4];
    __shared__ int sbin[TS];
    __shared__ float sl[TS];
    for (int k = threadIdx.x; k < NPARAM; k += 256) w[k] = prm[k];
    __syncthreads();
    const int t = threadIdx.x;
    if (t < TS) {
        const int64_t si = base + (int64_t)blockIdx.x * TS + t;
        float x[27], h1[32], h2[32], o[3], d[3];
        float tg[3];
        int b = 0;
        const bool valid = si < n;
        if (valid) {
            const Sample s = smp[si];
#pragma unroll
            for (int k = 0; k < 27; ++k) x[k] = (float)s.f[k] * (1.0f / 128.0f);
            b = s.bin;
#pragma unroll
            for (int c = 0; c < 3; ++c) tg[c] = (float)s.m[c] * (1.0f / 256.0f);
        } else {
#pragma unroll
            for (int k = 0; k < 27; ++k) x[k] = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) tg[c] = 0.0f;
        }
        for (int j = 0; j < 32; ++j) {
            float a = w[P_B1 + b * 32 + j];
            for (int k = 0; k < 27; ++k) a += w[P_W1 + j * 27 + k] * x[k];
            h1[j] = a;
        }
        for (int j = 0; j < 32; ++j) {
            float a = w[P_B2 + j];
            for (int k = 0; k < 32; ++k) a += w[P_W2 + j * 32 + k] * fmaxf(h1[k], 0.0f);
            h2[j] = a;
        }
        float loss = 0.0f;
        for (int c = 0; c < 3; ++c) {
            float a = w[P_B3 + c];
            for (int k = 0; k < 32; ++k) a += w[P_W3 + c * 32 + k] * fmaxf(h2[k], 0.0f);
            o[c] = a;
            const float e = a - tg[c];
            loss += valid ? e * e : 0.0f;
            d[c] = valid ? 2.0f * e * inv_count : 0.0f;
        }
        // backward
        float g2[32];
        for (int k = 0; k < 32; ++k) {
            float a = 0.0f;
            for (int c = 0; c < 3; ++c) a += w[P_W3 + c * 32 + k] * d[c];
            g2[k] = h2[k] > 0.0f ? a : 0.0f;
        }
        for (int k = 0; k < 32; ++k) {
            float a = 0.0f;
            for (int j = 0; j < 32; ++j) a += w[P_W2 + j * 32 + k] * g2[j];
            sd1[t][k] = h1[k] > 0.0f ? a : 0.0f;
        }
        for (int k = 0; k < 27; ++k) sx[t][k] = x[k];
        for (int k = 0; k < 32; ++k) {
            sa1[t][k] = fmaxf(h1[k], 0.0f);
            sa2[t][k] = fmaxf(h2[k], 0.0f);
            sd2[t][k] = g2[k];
        }
        for (int c = 0; c < 3; ++c) sdo[t][c] = d[c];
        sbin[t] = valid ? b : -1;
        sl[t] = loss;
    }
    __syncthreads();
    float *out = part + (int64_t)blockIdx.x * NPARAM;
    for (int p = threadIdx.x; p < NPARAM; p += 256) {
        float g = 0.0f;
        if (p < P_B1) {
            const int j = p / 27, k = p % 27;
            for (int s = 0; s < TS; ++s) g += sd1[s][j] * sx[s][k];
        } else if (p < P_W2) {
            const int b = (p - P_B1) / 32, j = (p - P_B1) % 32;
            for (int s = 0; s < TS; ++s) g += sbin[s] == b ? sd1[s][j] : 0.0f;
        } else if (p < P_B2) {
            const int j = (p - P_W2) / 32, k = (p - P_W2) % 32;
            for (int s = 0; s < TS; ++s) g += sd2[s][j] * sa1[s][k];
        } else if (p < P_W3) {
            const int j = p - P_B2;
            for (int s = 0; s < TS; ++s) g += sd2[s][j];
        } else if (p < P_B3) {
            const int c = (p - P_W3) / 32, k = (p - P_W3) % 32;
            for (int s = 0; s < TS; ++s) g += sdo[s][c] * sa2[s][k];
        } else {
            const int c = p - P_B3;
            for (int s = 0; s < TS; ++s) g += sdo[s][c];
        }
        out[p] = g;
    }
    if (threadIdx.x == 0) {
        float l = 0.0f;
        for (int s = 0; s < TS; ++s) l += sl[s];
        ploss[blockIdx.x] = l;
    }
}

// Sums the nwg partial gradients of each parameter in order and applies Adam.
// b1, b2 and their complements ob1 = 1 - b1, ob2 = 1 - b2 are the float32
// values nearest the exact ones (a complement taken in float32 from a rounded
// b2 = 0.999 would be off by 1.3e-5 relative); c1, c2 are the bias
// corrections 1 / (1 - b^step), also rounded once from their exact values.
__global__ __launch_bounds__(256) void k_train_adam(float *__restrict__ prm, float *__restrict__ m1, float *__restrict__ m2,
                                                    const float *__restrict__ part, const float *__restrict__ ploss,
                                                    int nwg, float lr, float b1, float b2, float ob1, float ob2,
                                                    float eps, float c1, float c2, float *__restrict__ loss_out) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < NPARAM) {
        float g = 0.0f;
        for (int k = 0; k < nwg; ++k) g += part[(int64_t)k * NPARAM + p];
        const float a = b1 * m1[p] + ob1 * g;
        const float v = b2 * m2[p] + ob2 * (g * g);
        m1[p] = a;
        m2[p] = v;
        prm[p] -= lr * (a * c1) / (sqrtf(v * c2) + eps);
    }
    if (p == 0 && loss_out) {
        float l = 0.0f;
        for (int k = 0; k < nwg; ++k) l += ploss[k];
        *loss_out = l;
    }
}

void launch_train_samples(const uint8_t *rgbe, const uint8_t *sdr, int H, int W, int k_img, const int64_t *idx,
                          int64_t n, void *out, hipStream_t s) {
    hipLaunchKernelGGL(k_train_samples, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rgbe, sdr, H, W, k_img,
                       idx, n, reinterpret_cast<Sample *>(out));
}

void launch_train_step(float *prm, float *m1, float *m2, const void *smp, int64_t base, int64_t nsamp, int batch,
                       float *part, float *ploss, float lr, int step, float *loss_out, hipStream_t s) {
    const int nwg = (batch + TS - 1) / TS;
    const int64_t avail = nsamp - base < batch ? nsamp - base : batch;
    const float inv = 1.0f / (3.0f * (float)(avail > 0 ? avail : 1));
    hipLaunchKernelGGL(k_train_grad, dim3(nwg), dim3(256), 0, s, prm, reinterpret_cast<const Sample *>(smp), base,
                       base + avail, inv, part, ploss);
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - pow(b1, step))), c2 = (float)(1.0 / (1.0 - pow(b2, step)));
    hipLaunchKernelGGL(k_train_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, prm, m1, m2, part, ploss, nwg, lr,
                       (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, c1, c2, loss_out);
}

int train_nparam() { return NPARAM; }
int train_sample_bytes() { return (int)sizeof(Sample); }

}  // namespace rdl
