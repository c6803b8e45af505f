// Orientation assignment and local descriptors on gfx950 (Sec. III-B and
// Sec. IV-B, Algorithm 2 stages A and B).
//
// One 64-lane wave (and workgroup) per keypoint.  The lanes
// sweep the bounding box of the keypoint's disk in row-major order (64
// pixels per step, the paper's pixel-level parallelism over a patch of
// variable size), and each in-disk pixel adds its weighted gradient to the
// wave's histogram in LDS with fixed-point integer atomics.  Peak finding, ranking and
// normalisation are wave-wide shuffles and ballots.
#include "cdvs_internal.h"

namespace cdvs {

namespace {

constexpr float kTwoPi = 6.283185307179586f;

// Sum over the wave, by the same row operations, swizzle and first-lane
// reads as the maximum below; every lane gets the same value.
__device__ __forceinline__ float wave_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xf, 0xf, false));    // xor 1
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xf, 0xf, false));    // xor 2
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xf, 0xf, false));   // half mirror
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xf, 0xf, false));   // mirror
    v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));                     // xor 16
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    return a + b;
}

// Maximum over the wave, by row operations (DPP) within each 16-lane row,
// a swizzle across row pairs and the two halves' first lanes.
__device__ __forceinline__ float wave_max_dpp(float v) {
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xf, 0xf, false)));  // xor 1
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xf, 0xf, false)));  // xor 2
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xf, 0xf, false))); // half mirror
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xf, 0xf, false))); // mirror
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F)));                    // xor 16
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    return fmaxf(a, b);
}

// q = n / d and r = n - q d for 0 <= n < 2^31, d >= 1: a single-precision
// estimate from the hardware reciprocal, refined once from the remainder
// (which leaves it at most one off) and corrected (products in unsigned
// arithmetic, so n - q d cannot overflow).
__device__ __forceinline__ void divmod_est(int n, int d, int& q, int& r) {
    const float inv = __builtin_amdgcn_rcpf((float)d);
    q = (int)((float)n * inv);
    r = (int)((unsigned)n - (unsigned)q * (unsigned)d);
    q += (int)((float)r * inv);
    r = (int)((unsigned)n - (unsigned)q * (unsigned)d);
    while (r < 0) {
        --q;
        r += d;
    }
    while (r >= d) {
        ++q;
        r -= d;
    }
}

// A keypoint the histogram kernels can take: octave in range, finite
// position, and a scale in octave units in (0, 2 sigma0] -- the largest a
// detected keypoint has (sigma* < sigma_4 = 2 sigma0), and the bound the
// host's fixed-point histogram scale is derived for, so that no bin can
// wrap.  Others get no orientation and an all-zero descriptor.
__device__ __forceinline__ bool keypoint_ok(const cdvs_keypoint& k, float sigma0) {
    if (k.octave < 0 || k.octave >= kMaxOctaves) return false;
    const float s = k.sigma * __builtin_amdgcn_ldexpf(1.0f, -k.octave);   // 2^-octave, exact
    return isfinite(k.x) && isfinite(k.y) && s > 0.f && s <= 2.f * sigma0;
}

// Squared distance of a pixel from the keypoint, as two rounded products
// and a rounded sum (never fused into a multiply-add): disk membership is a
// hard edge, and this way it is decided exactly as the plain definition
// computes it in single precision.
__device__ __forceinline__ float disk_d2(float dx, float dy) {
#pragma clang fp contract(off)
    return dx * dx + dy * dy;
}

struct KpGeom {
    const float* plane;  // G_{o,k*}
    int w, h, pitch;
    float cx, cy, s;     // octave pixels
};

// An empty statement that takes the keypoint count, record and octave-table
// entry as inputs: their loads are then all issued before it and waited for
// once, instead of each being sunk behind the branch that first uses it
// (three memory round trips in a row before the walk).
__device__ __forceinline__ void settle(int cnt, const cdvs_keypoint& k, const OctGeom& og) {
    asm volatile("" ::"v"(cnt), "v"(k.x), "v"(k.y), "v"(k.sigma), "v"(k.theta), "v"(k.octave), "v"(og.plane0),
                 "v"(og.w), "v"(og.h), "v"(og.pitch), "v"(og.plane_stride));
}

// og: this lane's entry of the keypoint's image's octave table (octave
// lane % 16), loaded beside the keypoint record; the keypoint's octave is
// the same in every lane, so its entry is read from that lane.
__device__ __forceinline__ int og_field(int v, int o) { return __builtin_amdgcn_readlane(v, o); }

__device__ __forceinline__ KpGeom keypoint_geometry(const float* pyr, const OctGeom& og, const cdvs_keypoint& k,
                                                    float sigma0) {
    KpGeom g;
    const int o = __builtin_amdgcn_readfirstlane(k.octave);
    const float sc = __builtin_amdgcn_ldexpf(1.0f, -k.octave);   // 2^-octave, exact
    g.cx = k.x * sc;
    g.cy = k.y * sc;
    g.s = k.sigma * sc;
    // nearest scale image: round(4 log2(s / sigma0)), clamped to 0..4
    const int ks = min(max((int)floorf(4.f * log2f(g.s / sigma0) + 0.5f), 0), kScales - 1);
    // one keypoint per wave: the plane pointer and pitch are the same in
    // every lane, and kept in scalar registers so that pixel addresses are
    // a 32-bit offset from them
    const int64_t plane0 = (int64_t)(((uint64_t)(uint32_t)og_field((int)(og.plane0 >> 32), o) << 32) |
                                     (uint32_t)og_field((int)og.plane0, o));
    const uint64_t po = (uint64_t)(plane0 + (int64_t)__builtin_amdgcn_readfirstlane(ks) * og_field(og.plane_stride, o));
    const uint32_t plo = __builtin_amdgcn_readfirstlane((uint32_t)po);
    const uint32_t phi = __builtin_amdgcn_readfirstlane((uint32_t)(po >> 32));
    g.plane = pyr + (int64_t)(((uint64_t)phi << 32) | plo);
    g.w = og_field(og.w, o);
    g.h = og_field(og.h, o);
    g.pitch = og_field(og.pitch, o);
    return g;
}

// Angle of (x, y) in [0, 2 pi], 2 pi itself only by rounding for angles
// just below it (both histograms take their bin index modulo the bin
// count, so 2 pi falls into bin 0 as 0 does).  The octant symmetries of
// the arctangent reduce the argument to t = min(|x|, |y|) / max(|x|, |y|)
// in [0, 1] (its rounding, under 2 ulp, moves the angle by less than
// 1e-7 rad), where
// atan(t) is an odd polynomial t P(t^2) of degree 11 whose coefficients are
// a minimax fit (Lawson's reweighted least squares on Chebyshev nodes of
// [0, 1], written by fit_atan_poly.py beside this file); its error is
// 1.7e-6 rad (2e-6 of a descriptor bin, 1e-5 of an orientation bin, whose
// linear split makes every pixel's contribution continuous in the angle),
// and the reflections add at most about one fp32 ulp of 2 pi (4.8e-7).
// (Degree 15 reached 6.7e-8 rad for two more multiply-adds per pixel.)
// (0, 0) gives 0.
__device__ __forceinline__ float angle_2pi(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    // mx is kept at least the smallest normal float, so (0, 0) gives
    // t = 0 * finite = 0 with no test
    const float mx = fmaxf(fmaxf(ax, ay), 1.17549435e-38f), mn = fminf(ax, ay);
    // mn / mx by the hardware reciprocal (1 ulp) and a multiply: a plain
    // division is a full IEEE sequence on this target, several times longer
    const float t = mn * __builtin_amdgcn_rcpf(mx);
    const float s = t * t;
    float p = -0.01171913556754589f;
    p = fmaf(p, s, 0.05264734849333763f);
    p = fmaf(p, s, -0.116426482796669f);
    p = fmaf(p, s, 0.19354037940502167f);
    p = fmaf(p, s, -0.33262282609939575f);
    p = fmaf(p, s, 0.9999772310256958f);
    float r = p * t;                                   // atan(t), in [0, pi/4]
    if (ay > ax) r = 1.5707963267948966f - r;          // first quadrant
    if (x < 0.f) r = 3.141592653589793f - r;           // upper half plane
    if (y < 0.f) r = kTwoPi - r;                       // lower half plane
    return r;
}

// The four neighbours of an interior pixel (u, v), and from them the
// gradient by central differences, angle in [0, 2 pi).
struct Nbrs {
    float l, r, d, u;   // (u-1, v), (u+1, v), (u, v-1), (u, v+1)
};

// (A 32-bit byte offset from the keypoint's plane base: one offset and two
// additions per pixel instead of four 64-bit addresses.  Row and pitch are
// below 2^24 (image sides are at most CDVS_MAX_SIDE), so the row offset is a
// full-rate 24-bit multiply.)
__device__ __forceinline__ Nbrs load_nbrs(const KpGeom& g, int u, int v) {
    const char* base = reinterpret_cast<const char*>(g.plane);
    const uint32_t off = (__umul24((uint32_t)v, (uint32_t)g.pitch) + (uint32_t)u) * 4u, dy = 4u * (uint32_t)g.pitch;
    return Nbrs{*reinterpret_cast<const float*>(base + (off - 4u)), *reinterpret_cast<const float*>(base + (off + 4u)),
                *reinterpret_cast<const float*>(base + (off - dy)), *reinterpret_cast<const float*>(base + (off + dy))};
}

__device__ __forceinline__ void gradient(const Nbrs& n, float& mag, float& ang) {
    const float gx = n.r - n.l;
    const float gy = n.u - n.d;
    mag = __builtin_amdgcn_sqrtf(gx * gx + gy * gy);   // hardware square root (1 ulp)
    ang = angle_2pi(gy, gx);
}

// Histograms accumulate in LDS as unsigned fixed point with integer atomics:
// on gfx950 LDS float atomic adds run ~4.5x slower than integer ones, and
// integer sums do not depend on the order of the adds.  The scale (OriParams
// and DescParams .fix) is the largest power of two for which no bin can
// overflow 32 bits; the host derives it from the window radius (2^14 for the
// orientation window and 2^12 for the descriptor window at the defaults).
// Histogram copies per wave: lane l adds into copy l % kCopies; copies are
// staggered by one bank.
constexpr int kCopies = 8;

// Keypoints (waves) per workgroup.  Each wave owns its keypoint's histogram
// outright, so waves never wait for each other: wave_sync() only orders one
// wave's own LDS accesses.  One wave per workgroup measured fastest (a
// workgroup's resources are released only when its slowest keypoint, the
// one with the largest window, is done).
constexpr int kKpWaves = 1;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
// Orientation histogram copy: 36 bins plus bins 36 and 37, which take the
// shares of bins 0 and 1 that wrap around (from bin 35, and from an angle
// of 2 pi, which rounding can give), folded into bins 0 and 1 at the end,
// so no bin index is wrapped per pixel; the stride of 38 words starts the
// eight copies on eight different banks.
constexpr int kOriStride = kOriBins + 2;
// Descriptor histogram copy: 4 x 4 cells of 9 bins, bin 8 taking the share
// of orientation bin 0 that wraps around from bin 7 (folded into bin 0 at
// the end, which leaves every integer sum unchanged), so that the eight
// adds of one pixel sit at fixed offsets from one base address; plus one
// word so that copies start on different banks.
constexpr int kDescCellBins = 9;
constexpr int kDescStride = 16 * kDescCellBins + 1;

// Zeroes the N words (a multiple of 4) of a 16-byte-aligned LDS histogram
// with the wave's 64 lanes, 16 bytes per lane and store, fully unrolled.
template <int N>
__device__ __forceinline__ void wave_zero(uint32_t* h, int lane) {
    static_assert(N % 4 == 0, "whole 16-byte groups");
    uint4* q = reinterpret_cast<uint4*>(h);
#pragma unroll
    for (int r = 0; r < (N / 4 + 63) / 64; ++r) {
        const int j = lane + 64 * r;
        if (N / 4 % 64 == 0 || j < N / 4) q[j] = make_uint4(0u, 0u, 0u, 0u);
    }
}

// Walks the bounding box [u0, u0+bw) x [v0, ...) in row-major order, 64
// pixels per step, without integer division in the loop; a lane is past the
// box's last row exactly when its pixel index is past the box.
struct BoxWalk {
    int u, v, du, dv, u1;
    __device__ __forceinline__ BoxWalk(int lane, int u0, int v0, int bw) {
        int q, r;
        divmod_est(lane, bw, q, r);
        u = u0 + r;
        v = v0 + q;
        divmod_est(64, bw, dv, du);
        u1 = u0 + bw - 1;
    }
    __device__ __forceinline__ void next(int bw) {
        u += du;
        v += dv;
        if (u > u1) {
            u -= bw;
            ++v;
        }
    }
};

__global__ __launch_bounds__(64 * kKpWaves) void k_orient(const float* __restrict__ pyr, const OctGeom* __restrict__ geom,
                                                const cdvs_keypoint* __restrict__ kp,
                                                const int32_t* __restrict__ count, int n_images, OriParams op,
                                                cdvs_keypoint* __restrict__ ori, int32_t* __restrict__ ori_cnt) {
    __shared__ __align__(16) uint32_t hist[kKpWaves][kCopies * kOriStride];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // the slot is the same in every lane: taken apart in scalar registers
    const uint32_t slot = (uint32_t)__builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * kKpWaves + wave);
    const uint32_t qimg = kp_div_q(slot, op.kp_div);
    const int img = (int)qimg, i = (int)(slot - qimg * (uint32_t)op.kp_cap);
    if (img >= n_images) return;   // uniform over the wave
    // the count, the record and the image's octave table (one octave per
    // lane) load together: one memory round trip before the walk
    const int cnt = count[img];
    const cdvs_keypoint k = kp[(int64_t)img * op.kp_cap + i];
    const OctGeom og = geom[img * kMaxOctaves + (lane & (kMaxOctaves - 1))];
    settle(cnt, k, og);
    if (i >= cnt) return;   // uniform over the wave
    if (!keypoint_ok(k, op.sigma0)) {
        if (lane == 0) ori_cnt[(int64_t)img * op.kp_cap + i] = 0;
        return;
    }
    wave_zero<kCopies * kOriStride>(hist[wave], lane);
    wave_sync();

    {
        uint32_t* hc = &hist[wave][(lane & (kCopies - 1)) * kOriStride];
        const KpGeom g = keypoint_geometry(pyr, og, k, op.sigma0);
        const float R = op.radius * g.s;
        const float R2 = R * R;
        const float ws = op.wsigma * g.s;
        // Gaussian weight in fixed-point units: fix exp(-d^2 / (2 ws^2)) =
        // 2^(d^2 nid + log2 fix), fix being a power of two
        // (the hardware reciprocal, 1 ulp: these per-keypoint constants need
        // no correctly rounded division)
        const float nid = -1.4426950408889634f * __builtin_amdgcn_rcpf(2.f * ws * ws), lfix = op.lfix;
        const int u0 = max((int)ceilf(g.cx - R), 1), u1 = min((int)floorf(g.cx + R), g.w - 2);
        const int v0 = max((int)ceilf(g.cy - R), 1), v1 = min((int)floorf(g.cy + R), g.h - 2);
        const int bw = u1 - u0 + 1, bh = v1 - v0 + 1;
        if (bw > 0 && bh > 0) {
            BoxWalk bwk(lane, u0, v0, bw);
            for (; bwk.v <= v1; bwk.next(bw)) {   // row-major: past the box once v > v1
                const int u = bwk.u, v = bwk.v;
                const float dx = (float)u - g.cx, dy = (float)v - g.cy;
                const float d2 = disk_d2(dx, dy);
                if (!(d2 < R2)) continue;
                const Nbrs nb = load_nbrs(g, u, v);
                float mag, ang;
                gradient(nb, mag, ang);
                const float wt = mag * __builtin_amdgcn_exp2f(fmaf(d2, nid, lfix));
                const float fb = ang * ((float)kOriBins / kTwoPi);
                const float f0 = floorf(fb);
                const float fr = fb - f0;
                const int b0 = (int)f0;   // 0 .. 36 (36 only for an angle of 2 pi)
                atomicAdd(hc + b0, (uint32_t)(wt - wt * fr + 0.5f));
                atomicAdd(hc + b0 + 1, (uint32_t)(wt * fr + 0.5f));   // bins 36, 37 are bins 0, 1
            }
        }
    }
    wave_sync();

    auto bin = [&](int b) {
        uint32_t t = 0u;
#pragma unroll
        for (int c = 0; c < kCopies; ++c)
            t += hist[wave][c * kOriStride + b] + (b < 2 ? hist[wave][c * kOriStride + kOriBins + b] : 0u);
        return (float)t * op.inv_fix;
    };
    // every lane reads its bin and both neighbours from the summed copies
    const float hsum = lane < kOriBins ? bin(lane) : 0.f;
    const float hb = hsum;
    const float hl = __shfl(hsum, lane == 0 ? kOriBins - 1 : lane - 1);
    const float hr = __shfl(hsum, lane == kOriBins - 1 ? 0 : lane + 1);
    const float mx = wave_max_dpp(hb);
    const bool pk = lane < kOriBins && hb > hl && hb > hr && hb > op.peak * mx;
    const uint64_t pm = __ballot(pk);
    int rank = 0;
    for (uint64_t m = pm; m; m &= m - 1) {
        const int j = __ffsll((unsigned long long)m) - 1;
        const float hj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hb), j));   // j is uniform
        if (hj > hb || (hj == hb && j < lane)) ++rank;
    }
    const int64_t base = ((int64_t)img * op.kp_cap + i);
    if (pk && rank < op.max_ori) {
        // a peak's parabola has hl - 2 hb + hr < 0; the hardware reciprocal
        // (1 ulp) moves the offset by far less than the angle tolerance
        const float off = 0.5f * (hl - hr) * __builtin_amdgcn_rcpf(hl - 2.f * hb + hr);
        float t = ((float)lane + off) * kTwoPi / (float)kOriBins;
        if (t < 0.f) t += kTwoPi;
        if (t >= kTwoPi) t -= kTwoPi;
        cdvs_keypoint r = k;
        r.theta = t;
        r.peak = hb;
        ori[base * kMaxOri + rank] = r;
    }
    if (lane == 0) ori_cnt[base] = min(__popcll(pm), op.max_ori);
}

// Expand the per-keypoint orientation records of one image in input order
// and cut at `limit`.  One 1024-lane workgroup per image: each lane takes a
// contiguous run of keypoints (one while the image has at most 1024), the
// runs' record counts are prefix-summed by wave scans and one scan of the
// wave totals, and each lane then copies its run's records.
constexpr int kCompactThreads = 1024;

__global__ __launch_bounds__(kCompactThreads) void k_orient_compact(const cdvs_keypoint* __restrict__ ori,
                                                                    const int32_t* __restrict__ ori_cnt,
                                                                    const int32_t* __restrict__ count_in, int kp_cap,
                                                                    int limit, cdvs_keypoint* __restrict__ out,
                                                                    int32_t* __restrict__ count_out) {
    __shared__ int wsum[kCompactThreads / 64];
    const int img = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = min(max(count_in[img], 0), kp_cap);
    const int chunk = (n + kCompactThreads - 1) / kCompactThreads;
    const int beg = min(tid * chunk, n), end = min(beg + chunk, n);
    const int32_t* cnt = ori_cnt + (int64_t)img * kp_cap;
    int sum = 0;
    for (int i = beg; i < end; ++i) sum += cnt[i];
    // inclusive scan within the wave
    int incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        int w = lane < kCompactThreads / 64 ? wsum[lane] : 0;
#pragma unroll
        for (int off = 1; off < kCompactThreads / 64; off <<= 1) {
            const int v = __shfl_up(w, off);
            if (lane >= off) w += v;
        }
        if (lane < kCompactThreads / 64) wsum[lane] = w;   // inclusive over waves
    }
    __syncthreads();
    int pos = incl - sum + (wave > 0 ? wsum[wave - 1] : 0);   // exclusive prefix
    for (int i = beg; i < end && pos < limit; ++i) {
        const int c = cnt[i];
        for (int j = 0; j < c && pos + j < limit; ++j)
            out[(int64_t)img * kp_cap + pos + j] = ori[((int64_t)img * kp_cap + i) * kMaxOri + j];
        pos += c;
    }
    if (tid == kCompactThreads - 1) count_out[img] = min(wsum[kCompactThreads / 64 - 1], limit);
}

__global__ __launch_bounds__(64 * kKpWaves) void k_describe(const float* __restrict__ pyr, const OctGeom* __restrict__ geom,
                                                  const cdvs_keypoint* __restrict__ kp,
                                                  const int32_t* __restrict__ count, int n_images, DescParams dp,
                                                  float* __restrict__ desc) {
    __shared__ __align__(16) uint32_t hist[kKpWaves][kCopies * kDescStride];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // the slot is the same in every lane: taken apart in scalar registers
    const uint32_t slot = (uint32_t)__builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * kKpWaves + wave);
    const uint32_t qimg = kp_div_q(slot, dp.kp_div);
    const int img = (int)qimg, i = (int)(slot - qimg * (uint32_t)dp.kp_cap);
    if (img >= n_images) return;   // uniform over the wave
    // the count, the record and the image's octave table (one octave per
    // lane) load together: one memory round trip before the walk
    const int cnt = count[img];
    const cdvs_keypoint k = kp[(int64_t)img * dp.kp_cap + i];
    const OctGeom og = geom[img * kMaxOctaves + (lane & (kMaxOctaves - 1))];
    settle(cnt, k, og);
    if (i >= cnt) return;   // uniform over the wave
    if (!keypoint_ok(k, dp.sigma0)) {
        float* out = desc + (((int64_t)img * dp.kp_cap + i) * kDescDim);
        out[lane] = 0.f;
        out[lane + 64] = 0.f;
        return;
    }
    wave_zero<kCopies * kDescStride>(hist[wave], lane);
    wave_sync();

    {
        uint32_t* hc = &hist[wave][(lane & (kCopies - 1)) * kDescStride];
        const KpGeom g = keypoint_geometry(pyr, og, k, dp.sigma0);
        const float th = k.theta;
        // hardware sine and cosine: theta is in [0, 2 pi), where they are
        // accurate to ~1e-6, far below what the cell weights can resolve
        const float ct = __cosf(th), st = __sinf(th);
        const float R = dp.radius * g.s;
        const float R2 = R * R;
        // cell units (the per-keypoint constants below use the hardware
        // reciprocal, 1 ulp, instead of correctly rounded divisions)
        const float icw = __builtin_amdgcn_rcpf(dp.cell * g.s);
        // rotation by -theta and the scale to cell units in one 2 x 2 matrix,
        // the cell-grid centre (1.5, 1.5) added by the same multiply-adds
        const float cti = ct * icw, sti = st * icw;
        // theta in eighths of a turn
        const float th8 = th * (8.f / kTwoPi);
        const float ws = dp.wsigma * g.s;
        // Gaussian weight in fixed-point units: fix exp(-d^2 / (2 ws^2)) =
        // 2^(d^2 nid + log2 fix), fix being a power of two
        const float nid = -1.4426950408889634f * __builtin_amdgcn_rcpf(2.f * ws * ws), lfix = dp.lfix;
        const int u0 = max((int)ceilf(g.cx - R), 1), u1 = min((int)floorf(g.cx + R), g.w - 2);
        const int v0 = max((int)ceilf(g.cy - R), 1), v1 = min((int)floorf(g.cy + R), g.h - 2);
        const int bw = u1 - u0 + 1, bh = v1 - v0 + 1;
        if (bw > 0 && bh > 0) {
            BoxWalk bwk(lane, u0, v0, bw);
            for (; bwk.v <= v1; bwk.next(bw)) {   // row-major: past the box once v > v1
                const int u = bwk.u, v = bwk.v;
                const float dx = (float)u - g.cx, dy = (float)v - g.cy;
                const float d2 = disk_d2(dx, dy);
                if (!(d2 < R2)) continue;
                const Nbrs nb = load_nbrs(g, u, v);
                const float fx = fmaf(cti, dx, fmaf(sti, dy, 1.5f));    // cell units, grid from 0
                const float fy = fmaf(cti, dy, fmaf(-sti, dx, 1.5f));
                float mag, ang;
                gradient(nb, mag, ang);
                const float wt = mag * __builtin_amdgcn_exp2f(fmaf(d2, nid, lfix));
                // Orientation relative to theta in eighths of a turn: ang - th
                // lies in (-2 pi, 2 pi], and the bin is floor(fo) modulo 8
                // (a mask by 7, right for either sign), so no wrap is needed.
                const float fo = fmaf(ang, 8.f / kTwoPi, -th8);
                const float o0f = floorf(fo);
                const float ao = fo - o0f, bo = 1.f - ao;
                const int o0 = (int)o0f & 7;
                // The two cells per axis are slots 0 and 1 from a base cell
                // clamped to 0..2.  Cell c's trilinear weight along an axis is
                // max(0, 1 - |f - c|): the usual 1 - a and a for the two cells
                // around f, 0 for any other, so a base shifted by the clamp, or
                // a cell outside the 4 x 4 grid, gets exactly its share.
                const float cx0 = __builtin_amdgcn_fmed3f(floorf(fx), 0.f, 2.f);
                const float cy0 = __builtin_amdgcn_fmed3f(floorf(fy), 0.f, 2.f);
                const float tx = fx - cx0, ty = fy - cy0;
                // (max(0, 1 - |t - 1|) is the median of t, 2 - t and 0)
                const float wx0 = fmaxf(0.f, 1.f - fabsf(tx));                    // base cell column
                const float wx1 = __builtin_amdgcn_fmed3f(tx, 2.f - tx, 0.f);     // the column after it
                const float wy0 = fmaxf(0.f, 1.f - fabsf(ty));
                const float wy1 = __builtin_amdgcn_fmed3f(ty, 2.f - ty, 0.f);
                // base cell's first bin: (4 by + bx) x 9, exact in float
                const int cell0 = (int)fmaf(cy0, 4.f * kDescCellBins, cx0 * (float)kDescCellBins);
                uint32_t* cell = hc + cell0 + o0;
#pragma unroll
                for (int jy = 0; jy < 2; ++jy) {
                    const float wy = wt * (jy ? wy1 : wy0);
#pragma unroll
                    for (int jx = 0; jx < 2; ++jx) {
                        const float wyx = wy * (jx ? wx1 : wx0);
                        uint32_t* c = cell + (jy * 4 + jx) * kDescCellBins;
                        atomicAdd(c, (uint32_t)fmaf(wyx, bo, 0.5f));      // rounded to nearest
                        atomicAdd(c + 1, (uint32_t)fmaf(wyx, ao, 0.5f));
                    }
                }
            }
        }
    }
    wave_sync();

    // element e = cell * 8 + bin; bin 0 also takes the cell's wrap bin
    uint32_t i0 = 0u, i1 = 0u;
    const int e0 = (lane >> 3) * kDescCellBins + (lane & 7), e1 = e0 + 8 * kDescCellBins;
    const bool wrap = (lane & 7) == 0;
#pragma unroll
    for (int c = 0; c < kCopies; ++c) {
        const uint32_t* h = &hist[wave][c * kDescStride];
        i0 += h[e0] + (wrap ? h[e0 + 8] : 0u);
        i1 += h[e1] + (wrap ? h[e1 + 8] : 0u);
    }
    const float h0 = (float)i0 * dp.inv_fix, h1 = (float)i1 * dp.inv_fix;
    float* out = desc + (((int64_t)img * dp.kp_cap + i) * kDescDim);
    const float n2 = wave_sum(h0 * h0 + h1 * h1);
    if (!(n2 > 0.f)) {
        out[lane] = 0.f;
        out[lane + 64] = 0.f;
        return;
    }
    // hardware reciprocal square roots (1 ulp; n2 > 0 and far from denormal)
    const float inv = __builtin_amdgcn_rsqf(n2);
    const float t0 = fminf(h0 * inv, dp.clamp), t1 = fminf(h1 * inv, dp.clamp);
    const float inv2 = __builtin_amdgcn_rsqf(wave_sum(t0 * t0 + t1 * t1));
    out[lane] = t0 * inv2;
    out[lane + 64] = t1 * inv2;
}

int blocks_for(int n_images, int kp_cap) {
    const int64_t waves = (int64_t)n_images * kp_cap;
    return (int)((waves + kKpWaves - 1) / kKpWaves);
}

}  // namespace

hipError_t launch_orient(const float* pyr, const OctGeom* geom, const cdvs_keypoint* kp, const int32_t* count,
                         int n_images, const OriParams& op, cdvs_keypoint* ori, int32_t* ori_cnt,
                         hipStream_t stream) {
    if (n_images <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_orient, dim3(blocks_for(n_images, op.kp_cap)), dim3(64 * kKpWaves), 0, stream, pyr, geom, kp, count,
                       n_images, op, ori, ori_cnt);
    return hipGetLastError();
}

hipError_t launch_orient_compact(const cdvs_keypoint* ori, const int32_t* ori_cnt, const int32_t* count_in,
                                 int n_images, int kp_cap, int topk, cdvs_keypoint* out, int32_t* count_out,
                                 hipStream_t stream) {
    if (n_images <= 0) return hipSuccess;
    const int limit = min(topk > 0 ? topk : kp_cap, kp_cap);
    hipLaunchKernelGGL(k_orient_compact, dim3(n_images), dim3(kCompactThreads), 0, stream, ori, ori_cnt, count_in, kp_cap,
                       limit, out, count_out);
    return hipGetLastError();
}

hipError_t launch_describe(const float* pyr, const OctGeom* geom, const cdvs_keypoint* kp, const int32_t* count,
                           int n_images, const DescParams& dp, float* desc, hipStream_t stream) {
    if (n_images <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_describe, dim3(blocks_for(n_images, dp.kp_cap)), dim3(64 * kKpWaves), 0, stream, pyr, geom, kp, count,
                       n_images, dp, desc);
    return hipGetLastError();
}

}  // namespace cdvs
