// Keypoint relevance and selection on gfx950 (Sec. III-B, Eqs. (4)-(5)):
// r = f1(sigma) f2(|p|) f3(d) f4(rho) f5(p_ss), each f a table over
// quantised values of one characteristic (bin = number of table edges at
// or below the value), and per image the keypoints of highest r are kept,
// equal r in their input order.  d is the distance to the image centre over
// the centre's distance to a corner.  Single precision, the products left
// to right, the distance without fused operations.
//
// One 1024-lane workgroup per image: every record's score is computed once,
// then (r, input index) pairs are sorted in LDS by a bitonic sort on 64-bit
// keys -- the complement of r's bits (r >= 0, so its bits order like its
// value) over the index -- and the first n_keep records are copied out.
#include "cdvs_internal.h"

namespace cdvs {

namespace {

constexpr int kRelThreads = 1024;

__device__ __forceinline__ float centre_distance(float x, float y, float hx, float hy) {
#pragma clang fp contract(off)
    const float dx = x - hx, dy = y - hy;
    return sqrtf(dx * dx + dy * dy) / sqrtf(hx * hx + hy * hy);
}

__device__ __forceinline__ int bin_of(const float* edges, float v) {
    int b = 0;
#pragma unroll
    for (int e = 0; e < kRelEdges; ++e) b += edges[e] <= v ? 1 : 0;
    return b;
}

__global__ __launch_bounds__(kRelThreads) void k_relevance(const cdvs_keypoint* __restrict__ kp_in,
                                                           const int32_t* __restrict__ count_in,
                                                           const int32_t* __restrict__ wh, int kp_cap,
                                                           const float* __restrict__ edges,
                                                           const float* __restrict__ values, int n_keep,
                                                           cdvs_keypoint* __restrict__ kp_out,
                                                           int32_t* __restrict__ count_out,
                                                           float* __restrict__ score_out) {
    __shared__ unsigned long long key[CDVS_MAX_KP_CAPACITY];
    __shared__ float se[kRelFeatures * kRelEdges], sv[kRelFeatures * kRelBins];
    const int img = blockIdx.x, tid = threadIdx.x;
    if (tid < kRelFeatures * kRelEdges) se[tid] = edges[tid];
    if (tid < kRelFeatures * kRelBins) sv[tid] = values[tid];
    __syncthreads();
    const int n = min(max(count_in[img], 0), kp_cap);
    int npow = 1;
    while (npow < n) npow <<= 1;
    const float hx = 0.5f * (float)(wh[2 * img] - 1), hy = 0.5f * (float)(wh[2 * img + 1] - 1);
    const cdvs_keypoint* in = kp_in + (int64_t)img * kp_cap;
    for (int i = tid; i < npow; i += kRelThreads) {
        unsigned long long k = ~0ull;   // padding sorts last
        if (i < n) {
            const cdvs_keypoint p = in[i];
            const float f[kRelFeatures] = {p.sigma, fabsf(p.p), centre_distance(p.x, p.y, hx, hy), p.rho, p.p_ss};
            float r = sv[bin_of(se, f[0])];
#pragma unroll
            for (int c = 1; c < kRelFeatures; ++c) r = r * sv[c * kRelBins + bin_of(se + c * kRelEdges, f[c])];
            k = ((unsigned long long)(0xFFFFFFFFu - __float_as_uint(r)) << 32) | (unsigned)i;
        }
        key[i] = k;
    }
    __syncthreads();
    for (int size = 2; size <= npow; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < npow; i += kRelThreads) {
                const int j = i ^ stride;
                if (j > i) {
                    const unsigned long long a = key[i], b = key[j];
                    const bool up = (i & size) == 0;
                    if ((a > b) == up) {
                        key[i] = b;
                        key[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    const int m = min(n, n_keep);
    for (int i = tid; i < m; i += kRelThreads) {
        const unsigned long long k = key[i];
        kp_out[(int64_t)img * kp_cap + i] = in[(unsigned)k];
        if (score_out) score_out[(int64_t)img * kp_cap + i] = __uint_as_float(0xFFFFFFFFu - (unsigned)(k >> 32));
    }
    if (tid == 0) count_out[img] = m;
}

}  // namespace

hipError_t launch_relevance(const cdvs_keypoint* kp_in, const int32_t* count_in, const int32_t* wh, int n_images,
                            int kp_cap, const float* edges, const float* values, int n_keep, cdvs_keypoint* kp_out,
                            int32_t* count_out, float* score_out, hipStream_t s) {
    if (n_images <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_relevance, dim3(n_images), dim3(kRelThreads), 0, s, kp_in, count_in, wh, kp_cap, edges, values,
                       n_keep, kp_out, count_out, score_out);
    return hipGetLastError();
}

}  // namespace cdvs
