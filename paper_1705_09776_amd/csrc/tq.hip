// Transform coding and ternary quantisation of local descriptors on gfx950
// (Sec. III-C): each 8-bin cell histogram goes through one of two order-8
// transforms of additions, subtractions and power-of-two scalings (cells
// with row + col even take set A, the others set B, so that neighbouring
// cells differ), and each transformed element is coded as -1, 0 or +1 by
// two thresholds of its own.  The first n elements of a priority order are
// packed at two bits each (01 = +1, 10 = -1, 00 = 0; position p in word
// p / 16, bits 2 (p % 16) and up) into eight 32-bit words per descriptor,
// so the code is 2n bits instead of the 512-byte float descriptor.
//
// One thread per (descriptor, cell), 16 descriptors per 256-lane
// workgroup.  Every transformed value is evaluated left to right as the
// transforms are written (parentheses first), in single precision, with no
// fused operations (there is no product to fuse; the scalings are exact),
// so the thresholds see exactly the values a plain single-precision
// evaluation gives.
#include "cdvs_internal.h"

namespace cdvs {

namespace {

constexpr int kTqDesc = 16;   // descriptors per workgroup

__global__ __launch_bounds__(256) void k_tq_encode(const float* __restrict__ desc, const int32_t* __restrict__ count,
                                                   int n_images, int kp_cap, const float* __restrict__ lo,
                                                   const float* __restrict__ hi, const int32_t* __restrict__ order,
                                                   int n_elem, uint32_t* __restrict__ codes) {
    __shared__ float slo[kDescDim], shi[kDescDim];
    __shared__ int sord[kDescDim];
    // symbol rows padded to 136 bytes: a cell's eight symbols go out as one
    // 8-byte store, and the four descriptors of a wave start on different banks
    constexpr int kSymStride = kDescDim + 8;
    __shared__ __align__(8) uint8_t sym[kTqDesc][kSymStride];
    const int tid = threadIdx.x, cell = tid & 15, dl = tid >> 4;
    if (tid < kDescDim) {
        slo[tid] = lo[tid];
        shi[tid] = hi[tid];
        sord[tid] = order[tid] & (kDescDim - 1);   // a position in the symbol row, whatever the caller passed
    }
    const int64_t g = (int64_t)blockIdx.x * kTqDesc + dl;
    const int img = (int)(g / kp_cap), i = (int)(g % kp_cap);
    const bool active = img < n_images && i < min(max(count[img], 0), kp_cap);
    __syncthreads();
    if (active) {
        const float4 a = *reinterpret_cast<const float4*>(desc + g * kDescDim + cell * 8);
        const float4 b = *reinterpret_cast<const float4*>(desc + g * kDescDim + cell * 8 + 4);
        const float h0 = a.x, h1 = a.y, h2 = a.z, h3 = a.w, h4 = b.x, h5 = b.y, h6 = b.z, h7 = b.w;
        float v[8];
        if ((((cell >> 2) + (cell & 3)) & 1) == 0) {   // set A
            v[0] = (h2 - h6) / 2.f;
            v[1] = (h3 - h7) / 2.f;
            v[2] = (h0 - h1) / 2.f;
            v[3] = (h2 - h3) / 2.f;
            v[4] = (h4 - h5) / 2.f;
            v[5] = (h6 - h7) / 2.f;
            v[6] = ((h0 + h4) - (h2 + h6)) / 4.f;
            v[7] = ((h0 + h2 + h4 + h6) - (h1 + h3 + h5 + h7)) / 8.f;
        } else {                                        // set B
            v[0] = (h0 - h4) / 2.f;
            v[1] = (h1 - h5) / 2.f;
            v[2] = (h7 - h0) / 2.f;
            v[3] = (h1 - h2) / 2.f;
            v[4] = (h3 - h4) / 2.f;
            v[5] = (h5 - h6) / 2.f;
            v[6] = ((h1 + h5) - (h3 + h7)) / 4.f;
            v[7] = ((h0 + h1 + h2 + h3) - (h4 + h5 + h6 + h7)) / 8.f;
        }
        uint32_t s0 = 0u, s1 = 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = cell * 8 + k;
            const uint32_t c = v[k] > shi[e] ? 1u : (v[k] < slo[e] ? 2u : 0u);
            if (k < 4) s0 |= c << (8 * k);
            else s1 |= c << (8 * (k - 4));
        }
        *reinterpret_cast<uint2*>(&sym[dl][cell * 8]) = make_uint2(s0, s1);
    }
    __syncthreads();
    if (active && cell < 8) {
        uint32_t w = 0u;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int p = cell * 16 + j;
            if (p < n_elem) w |= (uint32_t)sym[dl][sord[p]] << (2 * j);
        }
        codes[g * 8 + cell] = w;
    }
}

}  // namespace

hipError_t launch_tq_encode(const float* desc, const int32_t* count, int n_images, int kp_cap, const float* lo,
                            const float* hi, const int32_t* order, int n_elem, uint32_t* codes, hipStream_t s) {
    const int64_t slots = (int64_t)n_images * kp_cap;
    if (slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tq_encode, dim3((unsigned)((slots + kTqDesc - 1) / kTqDesc)), dim3(256), 0, s, desc, count,
                       n_images, kp_cap, lo, hi, order, n_elem, codes);
    return hipGetLastError();
}

}  // namespace cdvs
