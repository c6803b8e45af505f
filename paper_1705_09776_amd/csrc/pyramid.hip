// Gaussian scale space on gfx950 (Sec. III-A, Eq. (1); Sec. IV-A,
// Algorithm 1 stage A and its final downsampling step).
//
// One 256-lane workgroup per output tile of one (image, octave) (tile shape
// autotuned for the scale kernel).  The vertical pass reads input columns
// straight from global memory (adjacent lanes = adjacent columns, so every
// load is a contiguous 256-byte row segment; the halo rows are L1/L2 hits),
// all of a thread's column windows (8 output rows plus halo; 16 for the
// pre-blur) before filtering any, and produces the column-filtered rows T_k
// of every scale at once into LDS.  The horizontal pass reads T_k from LDS
// and writes each output row with 16-byte non-temporal stores.  The scale
// kernel also writes the even samples of G_{o,4}, which is G_{o+1,0}, so no
// separate downsampling pass exists.
#include "cdvs_internal.h"

namespace cdvs {

namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// Radius of tap set k: 0 = input pre-blur, 1..4 = scale images.
__host__ __device__ constexpr int radius_of(int k) {
    return k == 0 ? kR0 : k == 1 ? kR1 : k == 2 ? kR2 : k == 3 ? kR3 : kR4;
}

// Column pass of tap set K over a register window of V + 2*HALO rows:
// out[r] = sum_{p=-R..R} g_K[p] * win[r + HALO + p], taps in order p = -R..R.
template <int K, int HALO, int V>
__device__ __forceinline__ void column_pass(const float (&win)[V + 2 * HALO], const Taps& taps, float (&out)[V]) {
    constexpr int R = radius_of(K);
#pragma unroll
    for (int r = 0; r < V; ++r) {
        float acc = 0.f;
#pragma unroll
        for (int p = -R; p <= R; ++p) acc = fmaf(taps.g[K][p + R], win[r + HALO + p], acc);
        out[r] = acc;
    }
}

// Column pass of all four scale tap sets (1..4) for output row r of the
// window, written to T[k][row]: the taps are symmetric, so each set is
// g[0] x_0 + sum_p g[p] (x_p + x_-p), and the pair sums, formed once, serve
// all four sets (49 operations per pixel instead of 70).
template <int HALO, int V, int CP, int TH>
__device__ __forceinline__ void column_pass_scales(const float (&win)[V + 2 * HALO], const Taps& taps, int row0,
                                                   int scol, float (*T)[TH][CP]) {
    static_assert(HALO >= kR4 && kR4 >= kR3 && kR3 >= kR2 && kR2 >= kR1, "radii");
#pragma unroll
    for (int r = 0; r < V; ++r) {
        const float c = win[r + HALO];
        float pr[kR4 + 1];
#pragma unroll
        for (int p = 1; p <= kR4; ++p) pr[p] = win[r + HALO + p] + win[r + HALO - p];
        float a1 = taps.g[1][kR1] * c, a2 = taps.g[2][kR2] * c, a3 = taps.g[3][kR3] * c, a4 = taps.g[4][kR4] * c;
#pragma unroll
        for (int p = 1; p <= kR4; ++p) {
            if (p <= kR1) a1 = fmaf(taps.g[1][kR1 + p], pr[p], a1);
            if (p <= kR2) a2 = fmaf(taps.g[2][kR2 + p], pr[p], a2);
            if (p <= kR3) a3 = fmaf(taps.g[3][kR3 + p], pr[p], a3);
            a4 = fmaf(taps.g[4][kR4 + p], pr[p], a4);
        }
        T[0][row0 + r][scol] = a1;
        T[1][row0 + r][scol] = a2;
        T[2][row0 + r][scol] = a3;
        T[3][row0 + r][scol] = a4;
    }
}

// Row pass of tap set K for outputs 8 cg .. 8 cg + 7 of one LDS row (row
// points at column 0 of the T buffer, whose column c is image column
// x0 - HALO + c).  (A row layout skewed against bank conflicts measured
// slower: its extra LDS cost a workgroup per CU.)
template <int K, int HALO>
__device__ __forceinline__ void row_pass(const float* row, int cg, const Taps& taps, float (&out)[8]) {
    constexpr int R = radius_of(K);
    const float* base = row + 8 * cg;
    float in[8 + 2 * R];
#pragma unroll
    for (int i = 0; i < 8 + 2 * R; ++i) in[i] = base[HALO - R + i];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        float acc = 0.f;
#pragma unroll
        for (int p = -R; p <= R; ++p) acc = fmaf(taps.g[K][p + R], in[c + R + p], acc);
        out[c] = acc;
    }
}

// Plane rows are written with non-temporal stores: a pass writes far more
// plane bytes than the caches hold, and streaming them out instead of
// leaving dirty lines to be evicted later keeps the caches for the reads
// (scale planes 0.660 -> 0.619 ms and detection, which reads them back,
// 0.507 -> 0.450 ms per 256 images; plain stores of the same values
// otherwise).
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store8(float* dst, int x0, int w, const float (&v)[8]) {
    if (x0 + 8 <= w) {
        const f32x4 a = {v[0], v[1], v[2], v[3]}, b = {v[4], v[5], v[6], v[7]};
        __builtin_nontemporal_store(a, reinterpret_cast<f32x4*>(dst + x0));
        __builtin_nontemporal_store(b, reinterpret_cast<f32x4*>(dst + x0) + 1);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (x0 + i < w) dst[x0 + i] = v[i];
    }
}

// Even samples of 8 outputs starting at even column x0 -> 4 values at x0/2.
__device__ __forceinline__ void store_decimated(float* dst, int x0, int nw, const float (&v)[8]) {
    const int d0 = x0 >> 1;
    if (d0 + 4 <= nw) {
        const f32x4 a = {v[0], v[2], v[4], v[6]};
        __builtin_nontemporal_store(a, reinterpret_cast<f32x4*>(dst + d0));
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (d0 + i < nw) dst[d0 + i] = v[2 * i];
    }
}

// KFIRST..KFIRST+NK-1 are the tap sets applied; U8 selects the octave-0
// pre-blur (input = u8 image, output = G_{0,0}); otherwise input = G_{o,0},
// outputs G_{o,1..4} and the decimated G_{o+1,0}.
template <int KFIRST, int NK, int HALO, bool U8, int VAR>
__global__ __launch_bounds__(256) void k_blur(const uint8_t* __restrict__ images, float* __restrict__ pyr,
                                              const OctJob* __restrict__ jobs, const int32_t* __restrict__ owner,
                                              Taps taps) {
    // column window: 8 output rows for the scale planes, 16 for the pre-blur
    // (its single radius-7 filter leaves room for the longer window; each
    // was the faster of 4, 8 and 16 rows)
    constexpr int TW = blur_tw(VAR), TH = blur_th(VAR), V = U8 ? 2 * kBlurV : kBlurV;
    static_assert(TH % V == 0 && TW % 8 == 0, "tile shape");
    constexpr int C = TW + 2 * HALO;
    constexpr int CP = C + 1;
    constexpr int NG = TH / V;
    __shared__ float T[NK][TH][CP];

    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const OctJob& job = jobs[owner[tile]];   // per-tile owner table: one load, no search
    const int lt = tile - job.tile0_blur[VAR];
    const int tx0 = (lt % job.tiles_x_blur[VAR]) * TW;
    const int ty0 = (lt / job.tiles_x_blur[VAR]) * TH;
    const int w = job.w, h = job.h;

    // Every column window this thread owns is loaded before any is filtered,
    // so a thread with two windows does not wait twice for memory (and the
    // workgroup's barrier does not wait for that second round trip).
    constexpr int NI = (C * NG + 255) / 256;   // windows per thread (256 lanes)
    float win[NI][V + 2 * HALO];
#pragma unroll
    for (int ii = 0; ii < NI; ++ii) {
        const int t = threadIdx.x + ii * 256;
        if (t >= C * NG) break;
        const int col = t % C, grp = t / C;
        const int gx = clampi(tx0 - HALO + col, 0, w - 1);
        const int gy0 = ty0 + grp * V - HALO;
        // A window inside the image (all but the top and bottom tiles) is
        // read with one 32-bit byte offset from the uniform plane base,
        // advanced by the pitch per row; edge windows clamp every row (a
        // 24-bit multiply: rows and pitches are below 2^24, and a plane's
        // bytes below 2^32, as sides are at most CDVS_MAX_SIDE).
        const bool inside = gy0 >= 0 && gy0 + V + 2 * HALO <= h;
        if constexpr (U8) {
            const uint8_t* base = images + job.src;
            if (inside) {
                uint32_t off = (uint32_t)(gy0 * job.src_pitch + gx);
#pragma unroll
                for (int r = 0; r < V + 2 * HALO; ++r, off += (uint32_t)job.src_pitch) win[ii][r] = (float)base[off];
            } else {
#pragma unroll
                for (int r = 0; r < V + 2 * HALO; ++r)
                    win[ii][r] = (float)base[__umul24((uint32_t)clampi(gy0 + r, 0, h - 1), (uint32_t)job.src_pitch) +
                                             (uint32_t)gx];
            }
        } else {
            const char* base = reinterpret_cast<const char*>(pyr + job.plane0);
            if (inside) {
                uint32_t off = (uint32_t)(gy0 * job.pitch + gx) * 4u;
#pragma unroll
                for (int r = 0; r < V + 2 * HALO; ++r, off += 4u * (uint32_t)job.pitch)
                    win[ii][r] = *reinterpret_cast<const float*>(base + off);
            } else {
#pragma unroll
                for (int r = 0; r < V + 2 * HALO; ++r)
                    win[ii][r] = *reinterpret_cast<const float*>(
                        base + (__umul24((uint32_t)clampi(gy0 + r, 0, h - 1), (uint32_t)job.pitch) + (uint32_t)gx) * 4u);
            }
        }
    }
#pragma unroll
    for (int ii = 0; ii < NI; ++ii) {
        const int t = threadIdx.x + ii * 256;
        if (t >= C * NG) break;
        const int col = t % C, grp = t / C;
        if constexpr (NK == 1) {
            float out[V];
            column_pass<KFIRST, HALO, V>(win[ii], taps, out);
#pragma unroll
            for (int r = 0; r < V; ++r) T[0][grp * V + r][col] = out[r];
        } else {
            static_assert(KFIRST == 1 && NK == 4, "the scale kernel applies tap sets 1..4");
            column_pass_scales<HALO, V, CP, TH>(win[ii], taps, grp * V, col, T);
        }
    }
    __syncthreads();

    for (int t = threadIdx.x; t < TH * (TW / 8); t += blockDim.x) {
        const int row = t / (TW / 8), cg = t % (TW / 8);
        const int gy = ty0 + row, gx0 = tx0 + cg * 8;
        if (gy >= h || gx0 >= w) continue;
        float out[8];
        if constexpr (U8) {
            row_pass<KFIRST, HALO>(&T[0][row][0], cg, taps, out);
            store8(pyr + job.plane0 + (int64_t)gy * job.pitch, gx0, w, out);
        } else {
            float* base = pyr + job.plane0 + (int64_t)gy * job.pitch;
            row_pass<KFIRST, HALO>(&T[0][row][0], cg, taps, out);
            store8(base + (int64_t)1 * job.plane_stride, gx0, w, out);
            row_pass<KFIRST + 1, HALO>(&T[1 % NK][row][0], cg, taps, out);
            store8(base + (int64_t)2 * job.plane_stride, gx0, w, out);
            row_pass<KFIRST + 2, HALO>(&T[2 % NK][row][0], cg, taps, out);
            store8(base + (int64_t)3 * job.plane_stride, gx0, w, out);
            row_pass<KFIRST + 3, HALO>(&T[3 % NK][row][0], cg, taps, out);
            store8(base + (int64_t)4 * job.plane_stride, gx0, w, out);
            if (job.next0 >= 0 && (gy & 1) == 0)
                store_decimated(pyr + job.next0 + (int64_t)(gy >> 1) * job.next_pitch, gx0, job.next_w, out);
        }
    }
}

}  // namespace

hipError_t launch_preblur(const uint8_t* images, float* pyr, const OctJob* jobs, const int32_t* owner, int ntiles,
                          const Taps& taps, hipStream_t stream) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_blur<0, 1, kR0, true, kPreblurVariant>), dim3(ntiles), dim3(256), 0, stream, images, pyr,
                       jobs, owner, taps);
    return hipGetLastError();
}

hipError_t launch_scales(float* pyr, const OctJob* jobs, const int32_t* owner, int ntiles, int variant,
                         const Taps& taps, hipStream_t stream) {
    if (ntiles <= 0) return hipSuccess;
    switch (variant) {
#define CASE(V)                                                                                                   \
    case V:                                                                                                       \
        hipLaunchKernelGGL((k_blur<1, 4, kMaxR, false, V>), dim3(ntiles), dim3(256), 0, stream, nullptr, pyr, jobs, \
                           owner, taps);                                                                          \
        break;
        CASE(0)
        CASE(1)
        CASE(2)
        CASE(3)
#undef CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace cdvs
