// Variation operators of the tensorized EMO algorithms (Supplementary
// Sec. S.I) and the gather of the selected rows (Eq. (13)).
//
//  k_sbx_pm   one thread per (pair row r, variable j), four variables at a time
//             where rows are 16-byte aligned: simulated binary crossover of rows
//             r and h + r (Eq. (S.6)-(S.7)), the children clipped to [l, u], then
//             polynomial mutation of both (Eq. (S.8)-(S.11)).  Float32 math with
//             the hardware base-2 logarithm and exponential for the powers: the
//             operator streams 28 bytes per pair and variable, and float32 keeps it
//             near the HBM rate.
//  k_gather   one work-group per selected row, 16-byte copies where aligned.
// The random draws are inputs (uniform in [0, 1)).
#include "common.h"
#include "prims.h"

namespace nsga3 {

// x^e for x >= 0, e > 0 (0^e = 0): 2^(e log2 x) on the transcendental unit.
__device__ __forceinline__ float powp(float x, float e) {
    return __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(x));
}

struct VarParams {
    float ec;       // 1 / (eta_c + 1)
    float eta;      // eta_m + 1
    float ieta;     // 1 / eta
};

__device__ __forceinline__ float pm_one(float x, float lo, float hi, float m, const VarParams &p) {
    x = fminf(fmaxf(x, lo), hi);
    const float D = hi - lo;
    // With a draw of exactly 0 (or 1) the step is -d1 (or d2): taken directly,
    // since (1 - d1)^eta can underflow float32 (its eta-th root would then be 0).
    // For any other draw 2m (or 2 - 2m) is at least 2^-24 and such a term is
    // below its rounding.
    float step;
    if (m <= 0.5f) {
        const float d1 = (x - lo) / D;
        const float a = 2.0f * m;
        step = a == 0.0f ? -d1 : powp(a + (1.0f - a) * powp(1.0f - d1, p.eta), p.ieta) - 1.0f;
    } else {
        const float d2 = (hi - x) / D;
        const float a = 2.0f - 2.0f * m;
        step = a == 0.0f ? d2 : 1.0f - powp(a + (2.0f * m - 1.0f) * powp(1.0f - d2, p.eta), p.ieta);
    }
    return x + step * D;
}

__device__ __forceinline__ void sbx_pm_one(float x1, float x2, float m, float lo, float hi, float m1,
                                           float m2, const VarParams &p, float &o1, float &o2) {
    const float B = m <= 0.5f ? powp(2.0f * m, p.ec) : powp(1.0f / (2.0f - 2.0f * m), p.ec);
    const float c1 = ((1.0f + B) * x1 + (1.0f - B) * x2) * 0.5f;
    const float c2 = ((1.0f - B) * x1 + (1.0f + B) * x2) * 0.5f;
    o1 = pm_one(c1, lo, hi, m1, p);
    o2 = pm_one(c2, lo, hi, m2, p);
}

__global__ void k_var_status(int32_t *status) {
    if (threadIdx.x == 0 && status) *status = 0;
}

// bounds must be finite with l < u (checked once per variable by row 0's threads)
__global__ __launch_bounds__(256) void k_sbx_pm(const float *__restrict__ X, int64_t h, int d,
                                                const float *__restrict__ lower,
                                                const float *__restrict__ upper, VarParams p,
                                                const float *__restrict__ r_sbx,
                                                const float *__restrict__ r_pm,
                                                float *__restrict__ out, int32_t *status, bool vec) {
    const int64_t per_row = vec ? d / 4 : d;
    const int64_t total = h * per_row;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / per_row;
        const int c = (int)(t - r * per_row);
        if (vec) {
            const int j = 4 * c;
            const float4 a = *reinterpret_cast<const float4 *>(X + r * d + j);
            const float4 b = *reinterpret_cast<const float4 *>(X + (h + r) * d + j);
            const float4 m = *reinterpret_cast<const float4 *>(r_sbx + r * d + j);
            const float4 m1 = *reinterpret_cast<const float4 *>(r_pm + r * d + j);
            const float4 m2 = *reinterpret_cast<const float4 *>(r_pm + (h + r) * d + j);
            const float4 lo = *reinterpret_cast<const float4 *>(lower + j);
            const float4 hi = *reinterpret_cast<const float4 *>(upper + j);
            float4 o1, o2;
            sbx_pm_one(a.x, b.x, m.x, lo.x, hi.x, m1.x, m2.x, p, o1.x, o2.x);
            sbx_pm_one(a.y, b.y, m.y, lo.y, hi.y, m1.y, m2.y, p, o1.y, o2.y);
            sbx_pm_one(a.z, b.z, m.z, lo.z, hi.z, m1.z, m2.z, p, o1.z, o2.z);
            sbx_pm_one(a.w, b.w, m.w, lo.w, hi.w, m1.w, m2.w, p, o1.w, o2.w);
            *reinterpret_cast<float4 *>(out + r * d + j) = o1;
            *reinterpret_cast<float4 *>(out + (h + r) * d + j) = o2;
            if (r == 0 && status) {
                const bool ok = isfinite(lo.x) && isfinite(hi.x) && lo.x < hi.x && isfinite(lo.y) &&
                                isfinite(hi.y) && lo.y < hi.y && isfinite(lo.z) && isfinite(hi.z) &&
                                lo.z < hi.z && isfinite(lo.w) && isfinite(hi.w) && lo.w < hi.w;
                if (!ok) atomicOr(status, 1);
            }
            const bool fin = isfinite(o1.x) && isfinite(o1.y) && isfinite(o1.z) && isfinite(o1.w) &&
                             isfinite(o2.x) && isfinite(o2.y) && isfinite(o2.z) && isfinite(o2.w);
            if (!fin && status) atomicOr(status, 1);
        } else {
            const int j = c;
            const float lo = lower[j], hi = upper[j];
            float o1, o2;
            sbx_pm_one(X[r * d + j], X[(h + r) * d + j], r_sbx[r * d + j], lo, hi, r_pm[r * d + j],
                       r_pm[(h + r) * d + j], p, o1, o2);
            out[r * d + j] = o1;
            out[(h + r) * d + j] = o2;
            if (r == 0 && status && !(isfinite(lo) && isfinite(hi) && lo < hi)) atomicOr(status, 1);
            if (!(isfinite(o1) && isfinite(o2)) && status) atomicOr(status, 1);
        }
    }
}

// status bit 1 -> NSGA3_E_NONFINITE, bit 2 -> NSGA3_E_INVALID
__global__ void k_var_status_final(int32_t *status) {
    if (threadIdx.x == 0 && status) {
        const int32_t v = *status;
        *status = (v & 2) ? NSGA3_E_INVALID : (v & 1) ? NSGA3_E_NONFINITE : NSGA3_OK;
    }
}

__global__ __launch_bounds__(256) void k_gather(const float *__restrict__ X, int64_t N, int d,
                                                const int32_t *__restrict__ idx, int64_t K,
                                                float *__restrict__ out, int32_t *status, bool vec) {
    for (int64_t q = blockIdx.x; q < K; q += gridDim.x) {
        const int32_t i = idx[q];
        if (i < 0 || (int64_t)i >= N) {
            if (threadIdx.x == 0 && status) atomicOr(status, 2);
            continue;
        }
        const float *src = X + (int64_t)i * d;
        float *dst = out + q * d;
        if (vec) {
            for (int j = threadIdx.x; j < d / 4; j += blockDim.x)
                reinterpret_cast<float4 *>(dst)[j] = reinterpret_cast<const float4 *>(src)[j];
        } else {
            for (int j = threadIdx.x; j < d; j += blockDim.x) dst[j] = src[j];
        }
    }
}

hipError_t run_sbx_pm(const float *X, int64_t n, int d, const float *lower, const float *upper,
                      double eta_c, double eta_m, const float *r_sbx, const float *r_pm, float *out,
                      int32_t *status, hipStream_t s) {
    const int64_t h = n / 2;
    VarParams p;
    p.ec = (float)(1.0 / (eta_c + 1.0));
    p.eta = (float)(eta_m + 1.0);
    p.ieta = (float)(1.0 / (eta_m + 1.0));
    hipLaunchKernelGGL(k_var_status, dim3(1), dim3(64), 0, s, status);
    // 16-byte accesses when every row starts on a 16-byte boundary
    auto al = [](const void *q) { return ((uintptr_t)q & 15u) == 0; };
    const bool vec = (d & 3) == 0 && al(X) && al(lower) && al(upper) && al(r_sbx) && al(r_pm) && al(out);
    const int64_t per_row = vec ? d / 4 : d;
    const int64_t total = h * per_row;
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_sbx_pm, dim3((unsigned)g), dim3(256), 0, s, X, h, d, lower, upper, p, r_sbx,
                       r_pm, out, status, vec);
    hipLaunchKernelGGL(k_var_status_final, dim3(1), dim3(64), 0, s, status);
    return hipGetLastError();
}

hipError_t run_gather(const float *X, int64_t N, int d, const int32_t *idx, int64_t K, float *out,
                      int32_t *status, hipStream_t s) {
    hipLaunchKernelGGL(k_var_status, dim3(1), dim3(64), 0, s, status);
    int64_t g = K < 65536 ? K : 65536;
    if (g < 1) g = 1;
    const bool vec = (d & 3) == 0 && ((uintptr_t)X & 15u) == 0 && ((uintptr_t)out & 15u) == 0;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)g), dim3(256), 0, s, X, N, d, idx, K, out, status, vec);
    hipLaunchKernelGGL(k_var_status_final, dim3(1), dim3(64), 0, s, status);
    return hipGetLastError();
}

}  // namespace nsga3
