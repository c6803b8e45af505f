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
// The sort's exchanges at distances below 128 stay inside one 128-key
// chunk, which one wave holds in registers (two keys per lane) and
// exchanges by lane shuffles; only the longer distances go through LDS
// with a workgroup barrier each.
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

// One compare-exchange of a bitonic stage of block size `size` at distance
// S < 64, for the key k of element i held by this lane, whose partner
// (i ^ S) is in lane ^ S: the lower index keeps the smaller key in an
// ascending block, the larger in a descending one (by selects, no branch).
template <int S>
__device__ __forceinline__ unsigned long long bitonic_lane_step(unsigned long long k, int i, int size) {
    const unsigned long long o = lane_xor64<S>(k);
    const bool want_min = ((i & size) == 0) == ((i & S) == 0);
    const unsigned long long mn = o < k ? o : k, mx = o < k ? k : o;
    return want_min ? mn : mx;
}

// The steps at distances below 128 of bitonic block sizes first..last, on
// the 128-key chunks of key[0 .. npow): each wave takes whole chunks, two
// keys per lane (elements c*128 + lane and c*128 + 64 + lane).
__device__ __forceinline__ void bitonic_chunk_steps(unsigned long long* key, int npow, int first, int last) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int c = wave; c < npow / 128; c += nw) {
        const int i0 = 128 * c + lane, i1 = i0 + 64;
        unsigned long long k0 = key[i0], k1 = key[i1];
        for (int size = first; size <= last; size <<= 1) {
            if (size >= 128) {   // distance 64: the lane's own pair, one direction for both
                const bool asc = (i0 & size) == 0;
                const unsigned long long lo = k0 < k1 ? k0 : k1, hi = k0 < k1 ? k1 : k0;
                k0 = asc ? lo : hi;
                k1 = asc ? hi : lo;
            }
#define CDVS_STEP(S)                                 \
    if (size > S) {                                  \
        k0 = bitonic_lane_step<S>(k0, i0, size);     \
        k1 = bitonic_lane_step<S>(k1, i1, size);     \
    }
            CDVS_STEP(32) CDVS_STEP(16) CDVS_STEP(8) CDVS_STEP(4) CDVS_STEP(2) CDVS_STEP(1)
#undef CDVS_STEP
        }
        key[i0] = k0;
        key[i1] = k1;
    }
}

// Ascending bitonic sort of key[0 .. npow) (npow a power of two, at least
// 128) by the whole workgroup: block sizes up to 128 entirely in
// registers, then for each larger size its distances of 128 and more
// through LDS (a barrier each) and the rest in registers.
__device__ void bitonic_sort_keys(unsigned long long* key, int npow) {
    bitonic_chunk_steps(key, npow, 2, 128);
    __syncthreads();
    for (int size = 256; size <= npow; size <<= 1) {
        for (int stride = size >> 1; stride >= 128; stride >>= 1) {
            for (int t = threadIdx.x; t < npow / 2; t += blockDim.x) {
                const int lo = 2 * t - (t & (stride - 1)), hi = lo + stride;
                const unsigned long long a = key[lo], b = key[hi];
                if ((a > b) == ((lo & size) == 0)) {
                    key[lo] = b;
                    key[hi] = a;
                }
            }
            __syncthreads();
        }
        bitonic_chunk_steps(key, npow, size, size);
        __syncthreads();
    }
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
    int npow = 128;   // the sort works on whole 128-key chunks (padding sorts last)
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
    bitonic_sort_keys(key, npow);
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
