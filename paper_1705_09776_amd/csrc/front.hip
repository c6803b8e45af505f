// Front end: every input image brought down to a longer side of at most
// kFrontLongSide (640) pixels before the scale space is built (Sec. III:
// the encoder first reduces the resolution so that the longer side is at
// most 640).
//
// Area averaging in exact integer arithmetic.  Along an axis of n input and
// m output pixels, input pixel i spans [i m, (i + 1) m) and output pixel j
// spans [j n, (j + 1) n) in units of 1 / (n m) of the image; their overlap
// is an integer, the output pixel's weighted sum N = sum over its
// footprint of overlap_x * overlap_y * I is an exact integer, and the u8
// output is the mean rounded half up, floor((2 N + W H) / (2 W H)).  An
// image whose longer side is at most 640 maps onto itself (every overlap
// is the whole pixel) and is copied.
//
// One wave per output row, lanes along the row; 32 workgroups of 4 waves
// per image stride over its rows.
#include "cdvs_internal.h"

namespace cdvs {

namespace {

constexpr int kFrontParts = 32;   // workgroups per image

__global__ __launch_bounds__(256) void k_front(const uint8_t* __restrict__ src,
                                               const cdvs_image_desc* __restrict__ sdesc,
                                               uint8_t* __restrict__ dst, const cdvs_image_desc* __restrict__ ddesc,
                                               int n, int32_t* __restrict__ flags) {
    const int img = blockIdx.x / kFrontParts, part = blockIdx.x % kFrontParts;
    if (img >= n) return;
    const cdvs_image_desc s = sdesc[img], d = ddesc[img];
    const int W = s.width, H = s.height;
    int wo = -1, ho = -1;
    if (W >= 1 && H >= 1 && W <= CDVS_MAX_SIDE && H <= CDVS_MAX_SIDE && s.pitch >= W && s.offset >= 0)
        front_size(W, H, &wo, &ho);
    if (wo != d.width || ho != d.height) {   // uniform over the workgroup
        if (part == 0 && threadIdx.x == 0) atomicOr(flags, kFlagFrontShape);
        return;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (W == 2 * wo && H == 2 * ho && ((s.offset | s.pitch | d.offset | d.pitch) & 7) == 0) {
        // An exact factor of 2 (e.g. 1280x960 -> 640x480): every overlap is
        // a whole source pixel, so N = wo ho S for the 2x2 sum S, W H =
        // 4 wo ho, and the rounded mean is (S + 2) / 4 -- the same integers
        // as below.  Each lane takes 4 outputs from 8 bytes of both source
        // rows (8-byte aligned: offsets and pitches are multiples of 8).
        for (int y = part * 4 + wave; y < ho; y += kFrontParts * 4) {
            const uint8_t* r0 = src + s.offset + (int64_t)(2 * y) * s.pitch;
            const uint8_t* r1 = r0 + s.pitch;
            uint8_t* orow = dst + d.offset + (int64_t)y * d.pitch;
            for (int x4 = 4 * lane; x4 < wo; x4 += 256) {
                if (x4 + 4 <= wo) {
                    const uint2 a = *reinterpret_cast<const uint2*>(r0 + 2 * x4);
                    const uint2 b = *reinterpret_cast<const uint2*>(r1 + 2 * x4);
                    uint32_t o = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint32_t wa = k < 2 ? a.x : a.y, wb = k < 2 ? b.x : b.y;
                        const int sh = 16 * (k & 1);
                        const uint32_t sum = ((wa >> sh) & 255u) + ((wa >> (sh + 8)) & 255u) +
                                             ((wb >> sh) & 255u) + ((wb >> (sh + 8)) & 255u);
                        o |= ((sum + 2u) >> 2) << (8 * k);
                    }
                    *reinterpret_cast<uint32_t*>(orow + x4) = o;
                } else {
                    for (int x = x4; x < wo; ++x) {
                        const uint32_t sum = r0[2 * x] + r0[2 * x + 1] + r1[2 * x] + r1[2 * x + 1];
                        orow[x] = (uint8_t)((sum + 2u) >> 2);
                    }
                }
            }
        }
        return;
    }
    const uint32_t WH = (uint32_t)W * (uint32_t)H;
    // 2 N + W H < 511 W H: 32-bit arithmetic while that stays below 2^32
    const bool narrow = (uint64_t)WH * 511u < (1ull << 32);
    for (int y = part * 4 + wave; y < ho; y += kFrontParts * 4) {
        const int ylo = y * H, yhi = ylo + H;              // footprint, scaled by ho
        const int k0 = ylo / ho, k1 = (yhi - 1) / ho;
        uint8_t* orow = dst + d.offset + (int64_t)y * d.pitch;
        for (int x = lane; x < wo; x += 64) {
            const int xlo = x * W, xhi = xlo + W;          // footprint, scaled by wo
            const int i0 = xlo / wo, i1 = (xhi - 1) / wo;
            uint64_t N = 0;
            for (int k = k0; k <= k1; ++k) {
                const uint32_t oy = (uint32_t)(min((k + 1) * ho, yhi) - max(k * ho, ylo));
                const uint8_t* row = src + s.offset + (int64_t)k * s.pitch;
                uint32_t acc = 0;                           // <= 255 W < 2^21
                for (int i = i0; i <= i1; ++i)
                    acc += (uint32_t)(min((i + 1) * wo, xhi) - max(i * wo, xlo)) * row[i];
                N += (uint64_t)oy * acc;
            }
            orow[x] = narrow ? (uint8_t)((2u * (uint32_t)N + WH) / (2u * WH))
                             : (uint8_t)((2ull * N + WH) / (2ull * WH));
        }
    }
}

}  // namespace

hipError_t launch_front(const uint8_t* src, const cdvs_image_desc* sdesc, uint8_t* dst,
                        const cdvs_image_desc* ddesc, int n, int32_t* flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_front, dim3((unsigned)n * kFrontParts), dim3(256), 0, s, src, sdesc, dst, ddesc, n, flags);
    return hipGetLastError();
}

}  // namespace cdvs
